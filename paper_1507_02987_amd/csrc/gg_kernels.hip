// GPU kernels of the indexed similar-sequence search (Genoogle, arXiv
// 1507.02987, Sections 2, 2.1 and 2.2), written for gfx950 (CDNA4, wave64).
//
// Work is batched: every kernel handles all queries of a wave at once, so one
// query is just a batch of one.  Nothing here is a dense contraction, so there is
// no MFMA: the gather and sort stages are bound by HBM bandwidth and the banded
// Smith-Waterman by the integer vector ALUs.
#include <algorithm>

#include "gg_internal.h"

namespace gg {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int32_t base_code(uint32_t ch)
{
    // Section 2: DNA {A,C,G,T} or RNA {A,C,G,U}, 2 bits per base; A=0 C=1 G=2 T=U=3
    switch (ch) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': case 'U': case 'u': return 3;
    default: return -1;
    }
}

__device__ __forceinline__ uint64_t shr64(uint64_t x, int n) { return n >= 64 ? 0ull : (x >> n); }
__device__ __forceinline__ uint64_t low_mask(int n) { return n >= 64 ? ~0ull : ((1ull << n) - 1ull); }

__device__ __forceinline__ int32_t floor_half(int32_t x) { return x >> 1; }  // arithmetic shift

// 2-bit packed data bank, first base most significant: base of global index g
// sits in word g / 16 at bits 30 - 2 (g % 16); the array has one spare word.
__device__ __forceinline__ int32_t db_base(const uint32_t *__restrict__ dbw, int64_t g)
{
    return (int32_t)((dbw[g >> 4] >> (30u - ((uint32_t)(g & 15) << 1))) & 3u);
}

// Code of the k bases starting at global index g (first base most significant),
// the same integer the query's window of those bases has.
__device__ __forceinline__ uint32_t db_window(const uint32_t *__restrict__ dbw, int64_t g,
                                              int32_t k)
{
    const int64_t w = g >> 4;
    const uint64_t x = ((uint64_t)dbw[w] << 32) | (uint64_t)dbw[w + 1];
    return (uint32_t)((x << ((uint32_t)(g & 15) << 1)) >> (64 - 2 * k));
}

// Code of the window of `span` bases at global index g under a spaced-seed mask
// (bit t set: base t kept; Section 2.1).  A mask of all ones is the plain window.
__device__ __forceinline__ uint32_t db_code(const uint32_t *__restrict__ dbw, int64_t g,
                                            int32_t span, uint32_t mask)
{
    if (span <= 16 && mask == (1u << span) - 1u) return db_window(dbw, g, span);
    uint32_t c = 0;
    for (int32_t t = 0; t < span; ++t)
        if ((mask >> t) & 1u) c = c * 4u + (uint32_t)db_base(dbw, g + t);
    return c;
}

// Exclusive scan over the 256 threads of a block; *total receives the block sum.
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T *total)
{
    __shared__ T s_w[kBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    T x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    T before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) {
        T t = s_w[i];
        if (i < w) before += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return before + x - v;
}

// Bitonic sort of n <= 65536 records in LDS, through an index array.
template <typename Rec, typename Less>
__device__ void lds_bitonic(const Rec *__restrict__ s_r, uint16_t *__restrict__ s_ix, uint32_t n,
                            Less less)
{
    uint32_t n2 = 1;
    while (n2 < n) n2 <<= 1;
    for (uint32_t i = threadIdx.x; i < n2; i += blockDim.x) s_ix[i] = (uint16_t)i;
    __syncthreads();
    auto before = [&](uint32_t a, uint32_t b) -> bool {  // a strictly before b
        if (a >= n) return false;
        if (b >= n) return true;
        if (less(s_r[a], s_r[b])) return true;
        if (less(s_r[b], s_r[a])) return false;
        return a < b;
    };
    for (uint32_t k = 2; k <= n2; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < n2; i += blockDim.x) {
                const uint32_t l = i ^ j;
                if (l > i) {
                    const uint32_t a = s_ix[i], b = s_ix[l];
                    const bool up = (i & k) == 0;
                    if (up ? before(b, a) : before(a, b)) {
                        s_ix[i] = (uint16_t)b;
                        s_ix[l] = (uint16_t)a;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------------ S0: index build
// Formatting (Section 2): the bank's bases packed 2 bits each, 16 to a word, first
// base most significant; a byte outside the alphabet sets *err.
__global__ void k_pack_bases(const uint8_t *__restrict__ ascii, int64_t total,
                             uint32_t *__restrict__ dbw, int64_t nwords, int32_t *__restrict__ err)
{
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwords;
         w += (int64_t)gridDim.x * blockDim.x) {
        uint32_t word = 0;
        bool bad = false;
        for (int b = 0; b < 16; ++b) {
            const int64_t g = w * 16 + b;
            if (g >= total) break;
            const int32_t c = base_code(ascii[g]);
            bad |= c < 0;
            word |= (uint32_t)(c < 0 ? 0 : c) << (30 - 2 * b);
        }
        dbw[w] = word;
        if (bad) atomicOr(err, 1);
    }
}

// Sequence of window w: the last s with woff[s] <= w (woff: windows before s).
__device__ __forceinline__ int32_t window_seq(const uint32_t *__restrict__ woff, int32_t n_seqs,
                                              uint32_t w)
{
    int32_t lo = 0, hi = n_seqs - 1;
    while (lo < hi) {
        const int32_t m = (lo + hi + 1) >> 1;
        if (woff[m] <= w) lo = m;
        else hi = m - 1;
    }
    return lo;
}

// Index (Section 2.1): every non-overlapping window of every sequence, in (seq,
// pos) order: its code (the sort key), its number (the value) and a count per code.
__global__ void k_window_keys(const uint32_t *__restrict__ dbw, const int64_t *__restrict__ seq_start,
                              const uint32_t *__restrict__ woff, int32_t n_seqs, uint32_t n_win,
                              int32_t span, uint32_t mask, uint64_t *__restrict__ keys,
                              uint32_t *__restrict__ vals, uint32_t *__restrict__ counts)
{
    for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < n_win;
         w += gridDim.x * blockDim.x) {
        const int32_t s = window_seq(woff, n_seqs, w);
        const int64_t g = seq_start[s] + (int64_t)(w - woff[s]) * span;
        const uint32_t code = db_code(dbw, g, span, mask);
        keys[w] = code;
        vals[w] = w;
        atomicAdd(&counts[code], 1u);
    }
}

// Postings in list order: window number -> (sequence, position).
__global__ void k_postings(const uint32_t *__restrict__ vals, uint32_t n_win,
                           const uint32_t *__restrict__ woff, int32_t n_seqs, int32_t span,
                           int2 *__restrict__ post)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_win;
         i += gridDim.x * blockDim.x) {
        const uint32_t w = vals[i];
        const int32_t s = window_seq(woff, n_seqs, w);
        post[i] = int2{s, (int32_t)((w - woff[s]) * (uint32_t)span)};
    }
}

// The paired base of an ASCII base on the other strand (A-T, C-G; U pairs with
// A); any other byte is returned unchanged, so packing still rejects it.
__device__ __forceinline__ uint8_t paired_base(uint8_t ch)
{
    switch (ch) {
    case 'A': case 'a': return 'T';
    case 'C': case 'c': return 'G';
    case 'G': case 'g': return 'C';
    case 'T': case 't': case 'U': case 'u': return 'A';
    default: return ch;
    }
}

// Reverse strand of every sequence: dst[start[s] + i] = pair of src[start[s] + n_s - 1 - i],
// with start and n_s from the forward sequence starts.  One block per sequence
// (grid-stride over sequences), its threads striding through the bases.
__global__ void k_reverse_strand(const uint8_t *__restrict__ src, const int64_t *__restrict__ start,
                                 int32_t n_seqs, uint8_t *__restrict__ dst)
{
    for (int32_t s = blockIdx.x; s < n_seqs; s += gridDim.x) {
        const int64_t lo = start[s], n = start[s + 1] - lo;
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
            dst[lo + i] = paired_base(src[lo + n - 1 - i]);
    }
}

// Repeat cutoff: kept[c] = length of list c (heads in off) if it is at most
// max_posting, else 0.
__global__ void k_cut_counts(const uint32_t *__restrict__ off, uint32_t ncode, uint32_t max_posting,
                             uint32_t *__restrict__ kept)
{
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < ncode;
         c += gridDim.x * blockDim.x) {
        const uint32_t len = off[c + 1] - off[c];
        kept[c] = len > max_posting ? 0u : len;
    }
}

// Postings of the kept lists only: window i of the code-sorted order (code keys[i])
// moves from its place in list c of the full heads (off) to the same place in
// list c of the kept heads (kept_off); windows of dropped lists are skipped.
__global__ void k_postings_cut(const uint32_t *__restrict__ vals, const uint64_t *__restrict__ keys,
                               uint32_t n_win, const uint32_t *__restrict__ woff, int32_t n_seqs,
                               int32_t span, const uint32_t *__restrict__ off,
                               const uint32_t *__restrict__ kept_off, uint32_t max_posting,
                               int2 *__restrict__ post)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_win;
         i += gridDim.x * blockDim.x) {
        const uint32_t c = (uint32_t)keys[i];
        if (off[c + 1] - off[c] > max_posting) continue;
        const uint32_t w = vals[i];
        const int32_t s = window_seq(woff, n_seqs, w);
        post[kept_off[c] + (i - off[c])] = int2{s, (int32_t)((w - woff[s]) * (uint32_t)span)};
    }
}

void launch_reverse_strand(const uint8_t *src, const int64_t *start, int32_t n_seqs, uint8_t *dst,
                           hipStream_t st)
{
    if (n_seqs <= 0) return;
    const uint32_t nb = std::min<uint32_t>((uint32_t)n_seqs, kMaxGrid);
    k_reverse_strand<<<nb, kBlock, 0, st>>>(src, start, n_seqs, dst);
}

void launch_cut_counts(const uint32_t *off, uint32_t ncode, uint32_t max_posting, uint32_t *kept,
                       hipStream_t st)
{
    const uint32_t nb = std::min<uint32_t>((ncode + kBlock - 1) / kBlock, kMaxGrid);
    k_cut_counts<<<nb, kBlock, 0, st>>>(off, ncode, max_posting, kept);
}

void launch_postings_cut(const uint32_t *vals, const uint64_t *keys, uint32_t n_win,
                         const uint32_t *woff, int32_t n_seqs, int32_t span, const uint32_t *off,
                         const uint32_t *kept_off, uint32_t max_posting, int2 *post, hipStream_t st)
{
    if (n_win == 0) return;
    const uint32_t nb = std::min<uint32_t>((n_win + kBlock - 1) / kBlock, kMaxGrid);
    k_postings_cut<<<nb, kBlock, 0, st>>>(vals, keys, n_win, woff, n_seqs, span, off, kept_off,
                                          max_posting, post);
}

void launch_pack_bases(const uint8_t *ascii, int64_t total, uint32_t *dbw, int64_t nwords,
                       int32_t *err, hipStream_t st)
{
    if (nwords <= 0) return;
    const int64_t nb = std::min<int64_t>((nwords + kBlock - 1) / kBlock, kMaxGrid);
    k_pack_bases<<<(uint32_t)nb, kBlock, 0, st>>>(ascii, total, dbw, nwords, err);
}

void launch_window_keys(const uint32_t *dbw, const int64_t *seq_start, const uint32_t *woff,
                        int32_t n_seqs, uint32_t n_win, int32_t span, uint32_t mask,
                        uint64_t *keys, uint32_t *vals, uint32_t *counts, hipStream_t st)
{
    if (n_win == 0) return;
    const uint32_t nb = std::min<uint32_t>((n_win + kBlock - 1) / kBlock, kMaxGrid);
    k_window_keys<<<nb, kBlock, 0, st>>>(dbw, seq_start, woff, n_seqs, n_win, span, mask, keys,
                                         vals, counts);
}

void launch_postings(const uint32_t *vals, uint32_t n_win, const uint32_t *woff, int32_t n_seqs,
                     int32_t span, int2 *post, hipStream_t st)
{
    if (n_win == 0) return;
    const uint32_t nb = std::min<uint32_t>((n_win + kBlock - 1) / kBlock, kMaxGrid);
    k_postings<<<nb, kBlock, 0, st>>>(vals, n_win, woff, n_seqs, span, post);
}

// ------------------------------------------------------------------ S1/S2: encode + count
// One thread per query base g of the batch: code the base (flagging bytes outside
// the alphabet), find its query, and if a whole window of k bases starts here,
// code the window (first base most significant) and count its postings.
__global__ __launch_bounds__(kBlock) void k_encode_kmers(
    const uint8_t *__restrict__ ascii, const int64_t *__restrict__ qoff, int32_t nq, int64_t T,
    int32_t span, uint32_t mask, const uint32_t *__restrict__ list_off, uint8_t *__restrict__ qcode,
    uint32_t *__restrict__ kcode, uint32_t *__restrict__ cnt, uint32_t *__restrict__ lhead,
    int32_t *__restrict__ qid, int32_t *__restrict__ err, const int32_t *__restrict__ bq)
{
    // the block's bases and the span after them, coded once in LDS; the block's
    // first and last queries found once (bq: the query of each block's first base,
    // so the next block's bounds this one's last)
    __shared__ uint8_t s_c[kBlock + 32];
    __shared__ int32_t s_q[2];
    const int64_t g0 = (int64_t)blockIdx.x * kBlock;
    if (bq) {
        if (threadIdx.x < 2) {
            const bool last = g0 + kBlock >= T;
            s_q[threadIdx.x] = threadIdx.x == 0 ? bq[blockIdx.x] : (last ? nq - 1 : bq[blockIdx.x + 1]);
        }
    } else if (threadIdx.x < 2) {
        const int64_t x = min(g0 + (int64_t)(threadIdx.x ? kBlock - 1 : 0), T - 1);
        int32_t lo = 0, hi = nq - 1;  // last query whose first base is <= x
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (qoff[mid] <= x) lo = mid;
            else hi = mid - 1;
        }
        s_q[threadIdx.x] = lo;
    }
    for (int32_t x = threadIdx.x; x < kBlock + 32; x += kBlock) {
        const int64_t gx = g0 + x;
        int32_t c = gx < T ? base_code(ascii[gx]) : 0;
        if (c < 0) {
            if (x < kBlock) atomicOr(err, 1);  // flagged by the base's own block
            c = 0;
        }
        s_c[x] = (uint8_t)c;
    }
    __syncthreads();
    const int64_t g = g0 + threadIdx.x;
    if (g >= T) return;
    qcode[g] = s_c[threadIdx.x];
    int32_t lo = s_q[0], hi = s_q[1];
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (qoff[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    qid[g] = lo;
    uint32_t code = 0, n = 0, head = 0;
    if (g + span <= qoff[lo + 1]) {
        for (int32_t t = 0; t < span; ++t)
            if ((mask >> t) & 1u) code = code * 4u + s_c[threadIdx.x + t];  // kept bases only
        head = list_off[code];
        n = list_off[code + 1] - head;
    }
    kcode[g] = code;
    cnt[g] = n;
    lhead[g] = head;
}

// bq[b] = the query holding base b * kBlock, for every encode block b: each
// non-empty query writes the blocks that start inside it.
__global__ void k_block_query(const int64_t *__restrict__ qoff, int32_t nq,
                              int32_t *__restrict__ bq)
{
    const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    for (int64_t b = (qoff[q] + kBlock - 1) / kBlock; b * kBlock < qoff[q + 1]; ++b)
        bq[b] = q;
}

void launch_encode_kmers(const uint8_t *ascii, const int64_t *qoff, int32_t nq, int64_t T,
                         int32_t span, uint32_t mask, const uint32_t *list_off, uint8_t *qcode,
                         uint32_t *kcode, uint32_t *cnt, uint32_t *lhead, int32_t *qid,
                         int32_t *err, int32_t *bq, hipStream_t st)
{
    if (T <= 0) return;
    const int64_t nb = (T + kBlock - 1) / kBlock;
    if (bq) k_block_query<<<(nq + kBlock - 1) / kBlock, kBlock, 0, st>>>(qoff, nq, bq);
    k_encode_kmers<<<dim3((uint32_t)nb), dim3(kBlock), 0, st>>>(ascii, qoff, nq, T, span, mask,
                                                                list_off, qcode, kcode, cnt, lhead,
                                                                qid, err, bq);
}

// ------------------------------------------------------------------ scans
// Per-tile sums, then a per-tile scan whose offset is the sum of the earlier tiles'
// sums.  Up to kScanFuse tiles, each tile adds the earlier sums up itself (they are
// few and cached); beyond that one block first scans the tile sums.
constexpr int64_t kScanFuse = 2048;

// Four or two values read or written by one 16-byte access at an address that is
// only aligned to the value size (global accesses need dword alignment only).
typedef uint32_t u32x4_a4 __attribute__((ext_vector_type(4), aligned(4)));
typedef uint64_t u64x2_a8 __attribute__((ext_vector_type(2), aligned(8)));

// v[0 .. kItems) = p[i0 .. i0 + kItems), zeros past n; 16-byte loads when the
// thread's kItems values are all in range.
template <typename T>
__device__ __forceinline__ void load_items(const T *__restrict__ p, int64_t i0, int64_t n,
                                           T (&v)[kItems])
{
    if (i0 + kItems <= n) {
        if constexpr (sizeof(T) == 4) {
#pragma unroll
            for (int r = 0; r < kItems / 4; ++r) {
                const u32x4_a4 x = *reinterpret_cast<const u32x4_a4 *>(p + i0 + 4 * r);
                v[4 * r] = x.x;
                v[4 * r + 1] = x.y;
                v[4 * r + 2] = x.z;
                v[4 * r + 3] = x.w;
            }
        } else {
#pragma unroll
            for (int r = 0; r < kItems / 2; ++r) {
                const u64x2_a8 x = *reinterpret_cast<const u64x2_a8 *>(p + i0 + 2 * r);
                v[2 * r] = x.x;
                v[2 * r + 1] = x.y;
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < kItems; ++r) v[r] = i0 + r < n ? p[i0 + r] : (T)0;
    }
}

template <typename T>
__device__ __forceinline__ void store_items(T *__restrict__ p, int64_t i0, int64_t n,
                                            const T (&v)[kItems])
{
    if (i0 + kItems <= n) {
        if constexpr (sizeof(T) == 4) {
#pragma unroll
            for (int r = 0; r < kItems / 4; ++r) {
                u32x4_a4 x;
                x.x = v[4 * r];
                x.y = v[4 * r + 1];
                x.z = v[4 * r + 2];
                x.w = v[4 * r + 3];
                *reinterpret_cast<u32x4_a4 *>(p + i0 + 4 * r) = x;
            }
        } else {
#pragma unroll
            for (int r = 0; r < kItems / 2; ++r) {
                u64x2_a8 x;
                x.x = v[2 * r];
                x.y = v[2 * r + 1];
                *reinterpret_cast<u64x2_a8 *>(p + i0 + 2 * r) = x;
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < kItems; ++r)
            if (i0 + r < n) p[i0 + r] = v[r];
    }
}

// Scans of n values in tiles of kTile: thread t of a tile holds values
// [t kItems, t kItems + kItems) of it (16-byte accesses, adjacent threads on
// adjacent 32-byte pieces).  k_scan_reduce sums each tile; one block scans the
// tile sums; k_scan_down scans each tile from its offset.  Up to kScanFuse tiles,
// each tile adds the earlier sums up itself (they are few and cached).
template <typename TI, typename TO>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const TI *__restrict__ in, int64_t n,
                                                        TO *__restrict__ partials)
{
    TI v[kItems];
    load_items<TI>(in, (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems, n, v);
    TO s = 0;
#pragma unroll
    for (int r = 0; r < kItems; ++r) s += (TO)v[r];
    TO tot;
    block_excl_scan<TO>(s, &tot);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// One block of kPartBlock threads scans the nb tile sums in place and stores the
// total at partials[nb].  A chunk of kPartBlock * kItems sums is read at once,
// kItems consecutive sums per thread, so a few hundred thousand tiles take a few
// chunks, each one round trip to memory.
constexpr int kPartBlock = 1024;

template <typename TO>
__global__ __launch_bounds__(kPartBlock) void k_scan_partials(TO *__restrict__ partials, int64_t nb)
{
    constexpr int kWaves = kPartBlock / 64;
    __shared__ TO s_w[kWaves];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    TO carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += (int64_t)kPartBlock * kItems) {
        const int64_t i0 = b0 + (int64_t)threadIdx.x * kItems;
        TO v[kItems];
        load_items<TO>(partials, i0, nb, v);
        TO sum = 0;
#pragma unroll
        for (int r = 0; r < kItems; ++r) sum += v[r];
        TO x = sum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const TO y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) s_w[w] = x;
        __syncthreads();
        TO before = 0, tot = 0;
#pragma unroll
        for (int i = 0; i < kWaves; ++i) {
            const TO t = s_w[i];
            if (i < w) before += t;
            tot += t;
        }
        TO run = carry + before + x - sum;
#pragma unroll
        for (int r = 0; r < kItems; ++r) {
            const TO t = v[r];
            v[r] = run;
            run += t;
        }
        store_items<TO>(partials, i0, nb, v);
        carry += tot;
        __syncthreads();  // s_w is rewritten by the next chunk
    }
    if (threadIdx.x == 0) partials[nb] = carry;
}

template <typename TI, typename TO, bool FUSED>
__global__ __launch_bounds__(kBlock) void k_scan_down(const TI *__restrict__ in, int64_t n,
                                                      const TO *__restrict__ partials,
                                                      TO *__restrict__ out, int64_t nb,
                                                      TO *__restrict__ total_copy)
{
    // FUSED: partials holds each earlier tile's sum; this tile's offset is their sum
    // (a single tile reads none)
    TO pre = 0, all = 0;
    if (FUSED) {
        TO p = 0;
        for (int64_t b = threadIdx.x; b < (int64_t)blockIdx.x; b += kBlock) p += partials[b];
        block_excl_scan<TO>(p, &pre);
    } else {
        pre = partials[blockIdx.x];
        all = partials[nb];
    }
    const int64_t i0 = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    TI v[kItems];
    load_items<TI>(in, i0, n, v);
    TO s = 0;
#pragma unroll
    for (int r = 0; r < kItems; ++r) s += (TO)v[r];
    TO tot;
    TO run = block_excl_scan<TO>(s, &tot) + pre;
    if (FUSED) all = pre + tot;
    TO o[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        o[r] = run;
        run += (TO)v[r];
    }
    store_items<TO>(out, i0, n, o);
    if (blockIdx.x == nb - 1 && threadIdx.x == 0) {
        out[n] = all;
        if (total_copy) *total_copy = all;
    }
}

size_t scan_partials_needed(int64_t n) { return (size_t)((n + kTile - 1) / kTile + 1); }

// out[0..n] = exclusive scan of in[0..n) and the total; the total also goes to
// *total_copy when given.  A single tile is one launch.
template <typename TI, typename TO>
static void scan_impl(const TI *in, TO *out, int64_t n, TO *partials, hipStream_t st,
                      TO *total_copy = nullptr)
{
    if (n <= 0) {
        (void)hipMemsetAsync(out, 0, sizeof(TO), st);
        if (total_copy) (void)hipMemsetAsync(total_copy, 0, sizeof(TO), st);
        return;
    }
    const int64_t nb = (n + kTile - 1) / kTile;
    if (nb > 1) k_scan_reduce<TI, TO><<<dim3((uint32_t)nb), dim3(kBlock), 0, st>>>(in, n, partials);
    if (nb <= kScanFuse) {
        k_scan_down<TI, TO, true><<<dim3((uint32_t)nb), dim3(kBlock), 0, st>>>(in, n, partials,
                                                                               out, nb, total_copy);
    } else {
        k_scan_partials<TO><<<1, kPartBlock, 0, st>>>(partials, nb);
        k_scan_down<TI, TO, false><<<dim3((uint32_t)nb), dim3(kBlock), 0, st>>>(
            in, n, partials, out, nb, total_copy);
    }
}

void launch_scan_u32_to_u64(const uint32_t *in, uint64_t *out, int64_t n, uint64_t *partials,
                            hipStream_t st)
{
    scan_impl<uint32_t, uint64_t>(in, out, n, partials, st);
}

void launch_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *partials,
                     hipStream_t st)
{
    scan_impl<uint32_t, uint32_t>(in, out, n, partials, st);
}

__global__ void k_query_totals(const uint64_t *__restrict__ hoff, const int64_t *__restrict__ qoff,
                               int32_t nq, uint64_t *__restrict__ qtot)
{
    const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nq) qtot[q] = hoff[qoff[q + 1]] - hoff[qoff[q]];
}

void launch_query_totals(const uint64_t *hoff, const int64_t *qoff, int32_t nq, uint64_t *qtot,
                         hipStream_t st)
{
    if (nq <= 0) return;
    k_query_totals<<<(nq + kBlock - 1) / kBlock, kBlock, 0, st>>>(hoff, qoff, nq, qtot);
}

// ------------------------------------------------------------------ S3: gather
// Per position of the wave: its first hit (relative to the wave), the index of its
// posting list's head, and the constant part of its hits' keys
// (q << sh_q) + ((bias - qpos) << sh_d) + qpos.
// A replayed wave (ctl given) takes its plan entry plan[*cursor] here, and block 0
// publishes it in ctl for the wave's later kernels (the cursor moves on at the
// wave's end).
__global__ void k_wave_prep(const uint64_t *__restrict__ hoff, const int64_t *__restrict__ qoff,
                            const uint32_t *__restrict__ lhead, const int32_t *__restrict__ qid,
                            int32_t qa, int64_t g0,
                            int64_t np, HitKeyLayout lay, uint32_t *__restrict__ hrel,
                            uint32_t *__restrict__ pbase, uint64_t *__restrict__ akey,
                            const WaveCtl *__restrict__ plan, const uint32_t *__restrict__ cursor,
                            WaveCtl *__restrict__ ctl, uint32_t *__restrict__ tile_pos)
{
    if (ctl) {
        const WaveCtl w = plan[*cursor];
        if (blockIdx.x == 0 && threadIdx.x == 0) *ctl = w;
        qa = w.qa;
        g0 = w.g0;
        np = w.np;
        lay = w.lay;
    }
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p > np) return;
    const uint64_t hb = hoff[g0];
    const uint64_t r0 = hoff[g0 + p] - hb;
    hrel[p] = (uint32_t)r0;
    if (p == np) return;
    if (tile_pos) {  // the position holding each gather tile's first hit
        const uint64_t r1 = hoff[g0 + p + 1] - hb;
        for (uint64_t t = (r0 + kTile - 1) / kTile; t * kTile < r1; ++t) tile_pos[t] = (uint32_t)p;
    }
    const int64_t g = g0 + p;
    const int32_t q = qid[g];
    const int32_t qpos = (int32_t)(g - qoff[q]);
    pbase[p] = lhead[g];
    const int sh_d = lay.bp, sh_q = lay.bp + lay.bd + lay.bs;
    const uint64_t qpart = sh_q >= 64 ? 0ull : ((uint64_t)(uint32_t)(q - qa) << sh_q);
    akey[p] = qpart + ((uint64_t)(uint32_t)(lay.bias - qpos) << sh_d) + (uint64_t)(uint32_t)qpos;
}

void launch_wave_prep(const uint64_t *hoff, const int64_t *qoff, const uint32_t *lhead,
                      const int32_t *qid, int32_t qa, int64_t g0, int64_t g1, HitKeyLayout lay,
                      uint32_t *hrel, uint32_t *pbase, uint64_t *akey, uint32_t *tile_pos,
                      hipStream_t st)
{
    const int64_t np = g1 - g0;
    const int64_t nb = (np + 1 + kBlock - 1) / kBlock;
    k_wave_prep<<<dim3((uint32_t)nb), dim3(kBlock), 0, st>>>(hoff, qoff, lhead, qid, qa, g0, np,
                                                             lay, hrel, pbase, akey, nullptr,
                                                             nullptr, nullptr, tile_pos);
}

void launch_wave_prep_ctl(const uint64_t *hoff, const int64_t *qoff, const uint32_t *lhead,
                          const int32_t *qid, int64_t np_cap, uint32_t *hrel, uint32_t *pbase,
                          uint64_t *akey, const WaveCtl *plan, const uint32_t *cursor,
                          WaveCtl *ctl, uint32_t *tile_pos, hipStream_t st)
{
    const int64_t nb = (np_cap + 1 + kBlock - 1) / kBlock;
    k_wave_prep<<<dim3((uint32_t)nb), dim3(kBlock), 0, st>>>(hoff, qoff, lhead, qid, 0, 0, 0,
                                                             HitKeyLayout{}, hrel, pbase, akey,
                                                             plan, cursor, ctl, tile_pos);
}

// ------------------------------------------------------------------ S3 by sequence range
// A query whose hits overflow the per-call budget is searched in pieces, each over
// a contiguous range of data-bank sequence ids.  Lists are in (seq, pos) order, so
// the postings of sequences below s are a prefix of each list, found by binary
// search.
__device__ __forceinline__ uint32_t seq_lower_bound(const int2 *__restrict__ post, uint32_t lo,
                                                    uint32_t hi, int32_t s)
{
    while (lo < hi) {
        const uint32_t m = lo + ((hi - lo) >> 1);
        if (post[m].x < s) lo = m + 1;
        else hi = m;
    }
    return lo;
}

// below[y] += hits of the query's positions [0, np) on sequences < bounds[y]
// (block row y of the grid; cnt[p] is the full list length of position p).
__global__ __launch_bounds__(kBlock) void k_range_counts(const uint32_t *__restrict__ kcode,
                                                         const uint32_t *__restrict__ cnt,
                                                         int64_t np,
                                                         const uint32_t *__restrict__ list_off,
                                                         const int2 *__restrict__ post,
                                                         const int32_t *__restrict__ bounds,
                                                         unsigned long long *__restrict__ below)
{
    const int32_t s = bounds[blockIdx.y];
    unsigned long long c = 0;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < np;
         p += (int64_t)gridDim.x * kBlock) {
        const uint32_t n = cnt[p];
        if (n == 0) continue;
        const uint32_t lo = list_off[kcode[p]];
        c += seq_lower_bound(post, lo, lo + n, s) - lo;
    }
    unsigned long long tot;
    block_excl_scan<unsigned long long>(c, &tot);
    if (threadIdx.x == 0 && tot) atomicAdd(&below[blockIdx.y], tot);
}

void launch_range_counts(const uint32_t *kcode, const uint32_t *cnt, int64_t np,
                         const uint32_t *list_off, const int2 *post, const int32_t *bounds,
                         int32_t nbounds, unsigned long long *below, hipStream_t st)
{
    if (np <= 0 || nbounds <= 0) return;
    const uint32_t gx = (uint32_t)std::min<int64_t>((np + kBlock - 1) / kBlock, 64);
    k_range_counts<<<dim3(gx, (uint32_t)nbounds), kBlock, 0, st>>>(kcode, cnt, np, list_off, post,
                                                                    bounds, below);
}

// Positions of one query restricted to sequences [s_lo, s_hi): per position the
// start and length of its sub-list, and the constant part of its hit keys (the
// query's index in the wave is 0).
__global__ void k_piece_prep(const uint32_t *__restrict__ kcode, const uint32_t *__restrict__ cnt,
                             int64_t np, const uint32_t *__restrict__ list_off,
                             const int2 *__restrict__ post, int32_t s_lo, int32_t s_hi,
                             HitKeyLayout lay, uint32_t *__restrict__ pcnt,
                             uint32_t *__restrict__ pbase, uint64_t *__restrict__ akey)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const uint32_t n = cnt[p];
    uint32_t a = 0, b = 0;
    if (n) {
        const uint32_t lo = list_off[kcode[p]];
        a = seq_lower_bound(post, lo, lo + n, s_lo);
        b = seq_lower_bound(post, a, lo + n, s_hi);
    }
    pbase[p] = a;
    pcnt[p] = b - a;
    const int32_t qpos = (int32_t)p;
    akey[p] = ((uint64_t)(uint32_t)(lay.bias - qpos) << lay.bp) + (uint64_t)(uint32_t)qpos;
}

void launch_piece_prep(const uint32_t *kcode, const uint32_t *cnt, int64_t np,
                       const uint32_t *list_off, const int2 *post, int32_t s_lo, int32_t s_hi,
                       HitKeyLayout lay, uint32_t *pcnt, uint32_t *pbase, uint64_t *akey,
                       hipStream_t st)
{
    if (np <= 0) return;
    k_piece_prep<<<(uint32_t)((np + kBlock - 1) / kBlock), kBlock, 0, st>>>(
        kcode, cnt, np, list_off, post, s_lo, s_hi, lay, pcnt, pbase, akey);
}

// Load-balanced over hits: block b owns hits [b*kTile, (b+1)*kTile) of the wave.
// Consecutive threads take consecutive hits, so reads of one posting run and the
// key writes are coalesced.  The owning position of hit j is the last p with
// hrel[p] <= j, searched in LDS when the tile spans few positions.
//
// MODE 0 writes key j to keys[j].  MODE 1 and 2 serve the bucketed grouping: a
// hit of query q on sequence s falls in bucket bb[q] + (s * nb[q]) >> bs, one of
// nb[q] equal slices of the sequence-id range, so buckets in index order are in
// (q, s) order.  MODE 1 counts hits per bucket; MODE 2 writes each key into its
// bucket (in no particular order inside it), reserving space per tile and bucket.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_gather(
    const uint32_t *__restrict__ hrel, const uint32_t *__restrict__ pbase,
    const uint64_t *__restrict__ akey, int64_t np, const int2 *__restrict__ post, uint32_t nhits,
    int sh_s, int sh_d, int sh_q, int bs, uint64_t *__restrict__ keys,
    const uint32_t *__restrict__ bb, const uint32_t *__restrict__ nbq,
    uint32_t *__restrict__ bcount, const uint32_t *__restrict__ boff,
    const WaveCtl *__restrict__ ctl, const uint32_t *__restrict__ tile_pos)
{
    __shared__ uint32_t s_h[kGatherCap + 1];
    __shared__ uint32_t s_bin[kBinCap];
    __shared__ int64_t s_lo, s_hi;
    __shared__ uint32_t s_b0, s_nbin;
    if (MODE == 0 && ctl) {
        np = ctl->np;
        nhits = ctl->H;
        sh_s = ctl->lay.bp + ctl->lay.bd;
        sh_d = ctl->lay.bp;
    }
    const uint32_t t0 = blockIdx.x * (uint32_t)kTile;
    if (t0 >= nhits) return;  // a graph's grid covers the largest wave
    const uint32_t t1 = min(t0 + (uint32_t)kTile, nhits);
    if (MODE == 0 && tile_pos) {
        // the preparation recorded where each tile starts: this tile's positions
        // run from there to where the next tile starts (a bound on the last one's)
        if (threadIdx.x == 0) {
            s_lo = tile_pos[t0 / kTile];
            s_hi = t1 < nhits ? (int64_t)tile_pos[t1 / kTile] : np - 1;
        }
    } else if (threadIdx.x == 0) {
        int64_t a = 0, b = np - 1;
        while (a < b) {
            const int64_t m = (a + b + 1) >> 1;
            if (hrel[m] <= t0) a = m;
            else b = m - 1;
        }
        s_lo = a;
        b = np - 1;
        while (a < b) {
            const int64_t m = (a + b + 1) >> 1;
            if (hrel[m] <= t1 - 1) a = m;
            else b = m - 1;
        }
        s_hi = a;
        if (MODE != 0) {
            const uint32_t qf = (uint32_t)shr64(akey[s_lo], sh_q), ql = (uint32_t)shr64(akey[a], sh_q);
            s_b0 = bb[qf];
            s_nbin = bb[ql] + nbq[ql] - bb[qf];
        }
    }
    __syncthreads();
    const int64_t lo = s_lo, hi = s_hi;
    const bool in_lds = (hi - lo + 2) <= (int64_t)(kGatherCap + 1);
    if (in_lds)
        for (int64_t p = lo + threadIdx.x; p <= hi + 1; p += blockDim.x) s_h[p - lo] = hrel[p];
    const uint32_t b0 = MODE != 0 ? s_b0 : 0;
    const bool bins = MODE != 0 && s_nbin <= (uint32_t)kBinCap;
    if (bins)
        for (uint32_t i = threadIdx.x; i < s_nbin; i += blockDim.x) s_bin[i] = 0;
    __syncthreads();
    uint64_t kk[kItems];
    uint32_t bk[kItems], rk[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const uint32_t j = t0 + r * kBlock + threadIdx.x;
        bk[r] = 0xffffffffu;
        if (j >= t1) continue;
        int64_t p;
        uint32_t first;
        if (in_lds) {
            int32_t a = 0, b = (int32_t)(hi - lo);
            while (a < b) {
                const int32_t m = (a + b + 1) >> 1;
                if (s_h[m] <= j) a = m;
                else b = m - 1;
            }
            p = lo + a;
            first = s_h[a];
        } else {
            int64_t a = lo, b = hi;
            while (a < b) {
                const int64_t m = (a + b + 1) >> 1;
                if (hrel[m] <= j) a = m;
                else b = m - 1;
            }
            p = a;
            first = hrel[a];
        }
        const int2 e = post[pbase[p] + (j - first)];
        const uint64_t ak = akey[p];
        const uint64_t key = ak + ((uint64_t)(uint32_t)e.x << sh_s) + ((uint64_t)(uint32_t)e.y << sh_d);
        if (MODE == 0) {
            keys[j] = key;
            continue;
        }
        const uint32_t q = (uint32_t)shr64(ak, sh_q);
        const uint32_t bkt = bb[q] + (uint32_t)(((uint64_t)(uint32_t)e.x * nbq[q]) >> bs);
        bk[r] = bkt;
        kk[r] = key;
        if (bins) {
            rk[r] = atomicAdd(&s_bin[bkt - b0], 1u);
        } else if (MODE == 1) {
            atomicAdd(&bcount[bkt], 1u);
        } else {
            keys[boff[bkt] + atomicAdd(&bcount[bkt], 1u)] = key;
        }
    }
    if (MODE == 0 || !bins) return;  // uniform
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < s_nbin; i += blockDim.x) {
        const uint32_t c = s_bin[i];
        if (MODE == 1) {
            if (c) atomicAdd(&bcount[b0 + i], c);
        } else {
            s_bin[i] = c ? atomicAdd(&bcount[b0 + i], c) : 0u;  // count -> reserved start
        }
    }
    if (MODE == 1) return;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kItems; ++r)
        if (bk[r] != 0xffffffffu) keys[boff[bk[r]] + s_bin[bk[r] - b0] + rk[r]] = kk[r];
}

void launch_gather(const uint32_t *hrel, const uint32_t *pbase, const uint64_t *akey,
                   int64_t npos, const int2 *post, uint32_t nhits, HitKeyLayout lay,
                   uint64_t *keys, const uint32_t *tile_pos, hipStream_t st)
{
    if (nhits == 0) return;
    const uint32_t nb = (nhits + kTile - 1) / kTile;
    k_gather<0><<<nb, kBlock, 0, st>>>(hrel, pbase, akey, npos, post, nhits, lay.bp + lay.bd,
                                       lay.bp, 64, 0, keys, nullptr, nullptr, nullptr, nullptr,
                                       nullptr, tile_pos);
}

void launch_gather_ctl(const uint32_t *hrel, const uint32_t *pbase, const uint64_t *akey,
                       const int2 *post, uint32_t hits_cap, uint64_t *keys, const WaveCtl *ctl,
                       const uint32_t *tile_pos, hipStream_t st)
{
    const uint32_t nb = std::max<uint32_t>(1, (hits_cap + kTile - 1) / kTile);
    k_gather<0><<<nb, kBlock, 0, st>>>(hrel, pbase, akey, 0, post, 0, 0, 0, 64, 0, keys, nullptr,
                                       nullptr, nullptr, nullptr, ctl, tile_pos);
}

void launch_gather_bucket(int mode, const uint32_t *hrel, const uint32_t *pbase,
                          const uint64_t *akey, int64_t npos, const int2 *post, uint32_t nhits,
                          HitKeyLayout lay, const uint32_t *bb, const uint32_t *nbq,
                          uint32_t *bcount, const uint32_t *boff, uint64_t *keys, hipStream_t st)
{
    if (nhits == 0) return;
    const uint32_t nb = (nhits + kTile - 1) / kTile;
    const int sh_q = lay.bp + lay.bd + lay.bs;
    if (mode == 1)
        k_gather<1><<<nb, kBlock, 0, st>>>(hrel, pbase, akey, npos, post, nhits, lay.bp + lay.bd,
                                           lay.bp, sh_q, lay.bs, keys, bb, nbq, bcount, boff,
                                           nullptr, nullptr);
    else
        k_gather<2><<<nb, kBlock, 0, st>>>(hrel, pbase, akey, npos, post, nhits, lay.bp + lay.bd,
                                           lay.bp, sh_q, lay.bs, keys, bb, nbq, bcount, boff,
                                           nullptr, nullptr);
}

// ------------------------------------------------------------------ S4+S5 per bucket
// One block per bucket: sort its keys in LDS (bitonic; keys are unique), then
// chain them as k_chain_* does.  Each thread takes a contiguous slice of the
// sorted bucket, so a scan of the per-thread run counts gives every run its rank
// in key order; the bucket's runs go to a range reserved with one atomic.
__device__ __forceinline__ bool chain_end_lds(const uint64_t *__restrict__ s_k, uint32_t n,
                                              uint32_t i, int bp, int32_t k, int32_t G,
                                              int32_t M, int32_t *qs_out)
{
    const uint64_t pmask = low_mask(bp);
    const uint64_t key = s_k[i];
    const uint64_t grp = key >> bp;
    const int32_t qp = (int32_t)(key & pmask);
    if (i + 1 < n) {
        const uint64_t nx = s_k[i + 1];
        if ((nx >> bp) == grp && (int32_t)(nx & pmask) - (qp + k) <= G) return false;
    }
    uint32_t j = i;
    int32_t qj = qp;
    while (j > 0) {
        const uint64_t pv = s_k[j - 1];
        if ((pv >> bp) != grp) break;
        const int32_t qv = (int32_t)(pv & pmask);
        if (qj - (qv + k) > G) break;
        --j;
        qj = qv;
    }
    *qs_out = qj;
    return qp + k - qj >= M;
}

// One wave per bucket: the wave sorts the bucket's unique keys in its own LDS
// slice (bitonic network, wave-scope ordering only, no block barrier), then
// chains them; a ballot prefix gives every kept run its rank in key order, and
// the bucket's runs go to a range reserved with one atomic.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(kBlock) void k_bucket_sort_chain(
    const uint64_t *__restrict__ keys, const uint32_t *__restrict__ boff, uint32_t nbk,
    HitKeyLayout lay, int32_t k, int32_t G, int32_t M, Cand *__restrict__ tmp, uint32_t cap,
    uint32_t *__restrict__ cursor, uint32_t *__restrict__ btmp, uint32_t *__restrict__ bcands,
    uint32_t *__restrict__ cand_per_q)
{
    __shared__ uint64_t s_all[kBlock / 64][kBucketCapMax];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t bkt = blockIdx.x * (kBlock / 64) + w;
    if (bkt >= nbk) return;  // whole wave
    uint64_t *__restrict__ s_k = s_all[w];
    const uint32_t a0 = boff[bkt], n = boff[bkt + 1] - a0;
    if (n == 0 || n > kBucketCapMax) {  // larger buckets never reach this kernel
        if (lane == 0) bcands[bkt] = 0;
        return;
    }
    uint32_t n2 = 1;
    while (n2 < n) n2 <<= 1;
    for (uint32_t i = lane; i < n2; i += 64) s_k[i] = i < n ? keys[a0 + i] : ~0ull;
    wave_lds_sync();
    for (uint32_t kk = 2; kk <= n2; kk <<= 1) {
        for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
            for (uint32_t i = lane; i < n2; i += 64) {
                const uint32_t l = i ^ j;
                if (l > i) {
                    const uint64_t x = s_k[i], y = s_k[l];
                    if ((x > y) == ((i & kk) == 0)) {
                        s_k[i] = y;
                        s_k[l] = x;
                    }
                }
            }
            wave_lds_sync();
        }
    }
    const uint64_t below = (1ull << lane) - 1ull;
    uint32_t tot = 0;
    for (uint32_t base = 0; base < n; base += 64) {
        int32_t qs;
        const uint32_t i = base + lane;
        const bool e = i < n && chain_end_lds(s_k, n, i, lay.bp, k, G, M, &qs);
        tot += (uint32_t)__popcll(__ballot(e));
    }
    if (tot == 0) {
        if (lane == 0) bcands[bkt] = 0;
        return;
    }
    uint32_t at = 0;
    if (lane == 0) {
        at = atomicAdd(cursor, tot);
        btmp[bkt] = at;
        bcands[bkt] = tot;
        const uint32_t q = (uint32_t)shr64(s_k[0] >> lay.bp, lay.bd + lay.bs);
        atomicAdd(&cand_per_q[q], tot);
    }
    at = __shfl(at, 0, 64);
    if (at + tot > cap) return;  // past cap: the caller grows the buffer and reruns
    for (uint32_t base = 0; base < n; base += 64) {
        int32_t qs = 0;
        const uint32_t i = base + lane;
        const bool e = i < n && chain_end_lds(s_k, n, i, lay.bp, k, G, M, &qs);
        const uint64_t m = __ballot(e);
        if (e) {
            const uint64_t key = s_k[i];
            const uint64_t grp = key >> lay.bp;
            Cand cd;
            cd.d = (int32_t)(grp & low_mask(lay.bd)) - lay.bias;
            cd.s = (int32_t)(shr64(grp, lay.bd) & low_mask(lay.bs));
            cd.q = (int32_t)shr64(grp, lay.bd + lay.bs);
            cd.qs = qs;
            cd.qe = (int32_t)(key & low_mask(lay.bp)) + k;
            tmp[at + (uint32_t)__popcll(m & below)] = cd;
        }
        at += (uint32_t)__popcll(m);
    }
}

// Buckets over kBucketCapMax keys (a long run puts all its hits on one diagonal):
// one block per listed bucket, bitonic over the whole block in dynamic LDS, then
// each thread chains a contiguous slice and a block scan orders the runs.
__global__ __launch_bounds__(kBlock) void k_bucket_sort_chain_big(
    const uint64_t *__restrict__ keys, const uint32_t *__restrict__ boff,
    const uint32_t *__restrict__ list, HitKeyLayout lay, int32_t k, int32_t G, int32_t M,
    Cand *__restrict__ tmp, uint32_t cap, uint32_t *__restrict__ cursor,
    uint32_t *__restrict__ btmp, uint32_t *__restrict__ bcands, uint32_t *__restrict__ cand_per_q)
{
    extern __shared__ uint64_t s_k[];
    __shared__ uint32_t s_at;
    const uint32_t bkt = list[blockIdx.x];
    const uint32_t a0 = boff[bkt], n = boff[bkt + 1] - a0;
    uint32_t n2 = 1;
    while (n2 < n) n2 <<= 1;
    for (uint32_t i = threadIdx.x; i < n2; i += blockDim.x) s_k[i] = i < n ? keys[a0 + i] : ~0ull;
    __syncthreads();
    for (uint32_t kk = 2; kk <= n2; kk <<= 1) {
        for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < n2; i += blockDim.x) {
                const uint32_t l = i ^ j;
                if (l > i) {
                    const uint64_t x = s_k[i], y = s_k[l];
                    if ((x > y) == ((i & kk) == 0)) {
                        s_k[i] = y;
                        s_k[l] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    const uint32_t per = (n + blockDim.x - 1) / blockDim.x;
    const uint32_t lo = min(n, threadIdx.x * per), hi = min(n, lo + per);
    uint32_t c = 0;
    for (uint32_t i = lo; i < hi; ++i) {
        int32_t qs;
        if (chain_end_lds(s_k, n, i, lay.bp, k, G, M, &qs)) ++c;
    }
    uint32_t tot;
    const uint32_t ex = block_excl_scan<uint32_t>(c, &tot);
    if (threadIdx.x == 0) {
        const uint32_t at = tot ? atomicAdd(cursor, tot) : 0u;
        s_at = at;
        btmp[bkt] = at;
        bcands[bkt] = tot;
        if (tot) atomicAdd(&cand_per_q[(uint32_t)shr64(s_k[0] >> lay.bp, lay.bd + lay.bs)], tot);
    }
    __syncthreads();
    const uint32_t base = s_at;
    if (tot == 0 || base + tot > cap) return;  // past cap: the caller grows the buffer and reruns
    uint32_t at = base + ex;
    for (uint32_t i = lo; i < hi; ++i) {
        int32_t qs;
        if (chain_end_lds(s_k, n, i, lay.bp, k, G, M, &qs)) {
            const uint64_t key = s_k[i];
            const uint64_t grp = key >> lay.bp;
            Cand cd;
            cd.d = (int32_t)(grp & low_mask(lay.bd)) - lay.bias;
            cd.s = (int32_t)(shr64(grp, lay.bd) & low_mask(lay.bs));
            cd.q = (int32_t)shr64(grp, lay.bd + lay.bs);
            cd.qs = qs;
            cd.qe = (int32_t)(key & low_mask(lay.bp)) + k;
            tmp[at++] = cd;
        }
    }
}

void launch_bucket_sort_chain_big(const uint64_t *keys, const uint32_t *boff,
                                  const uint32_t *list, uint32_t nlist, uint32_t max_bucket,
                                  HitKeyLayout lay, int32_t k, int32_t max_gap, int32_t min_len,
                                  Cand *tmp, uint32_t cap, uint32_t *cursor, uint32_t *btmp,
                                  uint32_t *bcands, uint32_t *cand_per_q, hipStream_t st)
{
    if (nlist == 0) return;
    uint32_t n2 = 1;
    while (n2 < max_bucket) n2 <<= 1;
    k_bucket_sort_chain_big<<<nlist, kBlock, n2 * sizeof(uint64_t), st>>>(
        keys, boff, list, lay, k, max_gap, min_len, tmp, cap, cursor, btmp, bcands, cand_per_q);
}

hipError_t setup_kernels()
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_bucket_sort_chain_big),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(kBucketBig * sizeof(uint64_t)));
}

void launch_bucket_sort_chain(const uint64_t *keys, const uint32_t *boff, uint32_t nbk,
                              uint32_t max_bucket, HitKeyLayout lay, int32_t k, int32_t max_gap,
                              int32_t min_len, Cand *tmp, uint32_t cap, uint32_t *cursor,
                              uint32_t *btmp, uint32_t *bcands, uint32_t *cand_per_q,
                              hipStream_t st)
{
    (void)max_bucket;
    if (nbk == 0) return;
    const uint32_t per = kBlock / 64;
    k_bucket_sort_chain<<<(nbk + per - 1) / per, kBlock, 0, st>>>(
        keys, boff, nbk, lay, k, max_gap, min_len, tmp, cap, cursor, btmp, bcands, cand_per_q);
}

// Runs of bucket b move from their reserved range to their rank in bucket order.
__global__ void k_compact_cands(const Cand *__restrict__ tmp, const uint32_t *__restrict__ btmp,
                                const uint32_t *__restrict__ bcands,
                                const uint32_t *__restrict__ coff, Cand *__restrict__ out)
{
    const uint32_t b = blockIdx.x;
    const uint32_t n = bcands[b], from = btmp[b], to = coff[b];
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) out[to + i] = tmp[from + i];
}

void launch_compact_cands(const Cand *tmp, const uint32_t *btmp, const uint32_t *bcands,
                          const uint32_t *coff, uint32_t nbk, Cand *out, hipStream_t st)
{
    if (nbk) k_compact_cands<<<nbk, 64, 0, st>>>(tmp, btmp, bcands, coff, out);
}

// ------------------------------------------------------------------ S3+S4+S5 by probing
// Data-bank windows start at multiples of k, so the hits that can share a run
// with hit (qpos, dpos) of query q on sequence s lie on the same diagonal at
// (qpos +- m k, dpos +- m k); the closest one chains iff its gap (m - 1) k <= G,
// i.e. m <= G / k + 1.  Such a hit exists exactly when the query window at
// qpos + m k and the data-bank window at dpos + m k have the same code.  Each
// hit probes both sides (all loads issued together) and is then a single-hit
// run, the first hit of a longer run, its last hit, or inside it.  Single-hit
// runs are final (kept when k >= M); first and last hits are stored as run
// bounds and paired per query after sorting.  No other hit is ever stored, and
// the runs are those of sorting all hits by (q, s, diag, qpos) and scanning them.
__global__ __launch_bounds__(kBlock) void k_probe(
    const uint32_t *__restrict__ hrel, const uint32_t *__restrict__ pbase, int64_t np,
    const int2 *__restrict__ post, uint32_t nhits, int64_t g0, const int32_t *__restrict__ qid,
    const int64_t *__restrict__ qoff, int32_t qa, const uint32_t *__restrict__ kcode,
    const uint32_t *__restrict__ kcnt, const uint32_t *__restrict__ dbw,
    const int64_t *__restrict__ seq_start, int32_t k,
    uint32_t mask, int32_t mmax, int32_t M, Cand *__restrict__ cands, uint32_t ccap,
    uint32_t *__restrict__ ccount, uint32_t *__restrict__ cand_per_q, Bound *__restrict__ bounds,
    uint32_t bcap, uint32_t *__restrict__ bcount, uint32_t *__restrict__ bound_per_q)
{
    __shared__ uint32_t s_h[kGatherCap + 1];
    __shared__ int64_t s_lo, s_hi;
    const uint32_t t0 = blockIdx.x * (uint32_t)kTile;
    const uint32_t t1 = min(t0 + (uint32_t)kTile, nhits);
    if (threadIdx.x == 0) {
        int64_t a = 0, b = np - 1;
        while (a < b) {
            const int64_t m = (a + b + 1) >> 1;
            if (hrel[m] <= t0) a = m;
            else b = m - 1;
        }
        s_lo = a;
        b = np - 1;
        while (a < b) {
            const int64_t m = (a + b + 1) >> 1;
            if (hrel[m] <= t1 - 1) a = m;
            else b = m - 1;
        }
        s_hi = a;
    }
    __syncthreads();
    const int64_t lo = s_lo, hi = s_hi;
    const bool in_lds = (hi - lo + 2) <= (int64_t)(kGatherCap + 1);
    if (in_lds)
        for (int64_t p = lo + threadIdx.x; p <= hi + 1; p += blockDim.x) s_h[p - lo] = hrel[p];
    __syncthreads();
    const int lane = threadIdx.x & 63;
#pragma unroll 2
    for (int r = 0; r < kItems; ++r) {
        const uint32_t j = t0 + r * kBlock + threadIdx.x;
        int kind = 0;  // 0 none, 1 single-hit run kept, 2 run bound
        int32_t q = 0, sq = 0, d = 0, qpos = 0;
        if (j < t1) {
            int64_t p;
            uint32_t first;
            if (in_lds) {
                int32_t a = 0, b = (int32_t)(hi - lo);
                while (a < b) {
                    const int32_t m = (a + b + 1) >> 1;
                    if (s_h[m] <= j) a = m;
                    else b = m - 1;
                }
                p = lo + a;
                first = s_h[a];
            } else {
                int64_t a = lo, b = hi;
                while (a < b) {
                    const int64_t m = (a + b + 1) >> 1;
                    if (hrel[m] <= j) a = m;
                    else b = m - 1;
                }
                p = a;
                first = hrel[a];
            }
            const int2 e = post[pbase[p] + (j - first)];
            const int64_t g = g0 + p;
            q = qid[g];
            const int64_t qb = qoff[q];
            const int32_t L = (int32_t)(qoff[q + 1] - qb);
            qpos = (int32_t)(g - qb);
            const int64_t s0 = seq_start[e.x];
            const int32_t ns = (int32_t)(seq_start[e.x + 1] - s0);
            // a neighbour window is a hit when its code equals the query window's
            // and that code's list is indexed (a repeat cutoff may have dropped it;
            // a kept list holds every window of its code, so it is not empty)
            bool pred = false, succ = false;
#pragma unroll
            for (int32_t m = 1; m <= kMaxProbe; ++m) {
                if (m > mmax) break;
                const int32_t qp = qpos - m * k, dp = e.y - m * k;
                if (qp >= 0 && dp >= 0 && kcnt[qb + qp] > 0u)
                    pred |= kcode[qb + qp] == db_code(dbw, s0 + dp, k, mask);
                const int32_t qn = qpos + m * k, dn = e.y + m * k;
                if (qn + k <= L && dn + k <= ns && kcnt[qb + qn] > 0u)
                    succ |= kcode[qb + qn] == db_code(dbw, s0 + dn, k, mask);
            }
            sq = e.x;
            d = e.y - qpos;
            if (!pred && !succ) kind = (k >= M) ? 1 : 0;
            else if (pred != succ) kind = 2;
        }
        const uint64_t m1 = __ballot(kind == 1);
        if (m1) {
            const int leader = __ffsll((unsigned long long)m1) - 1;
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(ccount, (uint32_t)__popcll(m1));
            base = __shfl(base, leader, 64);
            if (kind == 1) {
                const uint32_t at = base + (uint32_t)__popcll(m1 & ((1ull << lane) - 1ull));
                if (at < ccap) cands[at] = Cand{q - qa, sq, d, qpos, qpos + k};
                atomicAdd(&cand_per_q[q - qa], 1u);
            }
        }
        const uint64_t m2 = __ballot(kind == 2);
        if (m2) {
            const int leader = __ffsll((unsigned long long)m2) - 1;
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(bcount, (uint32_t)__popcll(m2));
            base = __shfl(base, leader, 64);
            if (kind == 2) {
                const uint32_t at = base + (uint32_t)__popcll(m2 & ((1ull << lane) - 1ull));
                if (at < bcap) bounds[at] = Bound{q - qa, sq, d, qpos};
                atomicAdd(&bound_per_q[q - qa], 1u);
            }
        }
    }
}

void launch_probe(const uint32_t *hrel, const uint32_t *pbase, int64_t np, const int2 *post,
                  uint32_t nhits, int64_t g0, const int32_t *qid, const int64_t *qoff, int32_t qa,
                  const uint32_t *kcode, const uint32_t *kcnt, const uint32_t *dbw,
                  const int64_t *seq_start, int32_t k,
                  uint32_t mask, int32_t max_gap, int32_t min_len, Cand *cands, uint32_t ccap,
                  uint32_t *ccount, uint32_t *cand_per_q, Bound *bounds, uint32_t bcap,
                  uint32_t *bcount, uint32_t *bound_per_q, hipStream_t st)
{
    // k is the window span here; mask picks its coded bases
    if (nhits == 0) return;
    const uint32_t nb = (nhits + kTile - 1) / kTile;
    k_probe<<<nb, kBlock, 0, st>>>(hrel, pbase, np, post, nhits, g0, qid, qoff, qa, kcode, kcnt, dbw,
                                   seq_start, k, mask, max_gap / k + 1, min_len, cands, ccap,
                                   ccount, cand_per_q, bounds, bcap, bcount, bound_per_q);
}

// Run bounds appended in any order go to their query's range (counting sort).
__global__ void k_bounds_by_query(const Bound *__restrict__ in, uint32_t n,
                                  const uint32_t *__restrict__ qoff_b, uint32_t *__restrict__ cur,
                                  Bound *__restrict__ out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Bound b = in[i];
    out[qoff_b[b.q] + atomicAdd(&cur[b.q], 1u)] = b;
}

void launch_bounds_by_query(const Bound *in, uint32_t n, const uint32_t *qoff_b, uint32_t *cur,
                            Bound *out, hipStream_t st)
{
    if (n) k_bounds_by_query<<<(n + kBlock - 1) / kBlock, kBlock, 0, st>>>(in, n, qoff_b, cur, out);
}

struct BoundLess {
    __device__ bool operator()(const Bound &x, const Bound &y) const
    {
        if (x.s != y.s) return x.s < y.s;
        if (x.d != y.d) return x.d < y.d;
        return x.qpos < y.qpos;
    }
};

// One block per query: sort its run bounds by (s, diag, qpos); they then
// alternate first hit, last hit, so pair 2i and 2i + 1 spans one run.
__global__ __launch_bounds__(kBlock) void k_pair_bounds(const Bound *__restrict__ b,
                                                        const uint32_t *__restrict__ qoff_b,
                                                        int32_t k, int32_t M,
                                                        Cand *__restrict__ cands, uint32_t ccap,
                                                        uint32_t *__restrict__ ccount,
                                                        uint32_t *__restrict__ cand_per_q)
{
    __shared__ Bound s_r[kBoundCap];
    __shared__ uint16_t s_ix[kBoundCap];
    const int32_t ql = blockIdx.x;
    const uint32_t a0 = qoff_b[ql], n = qoff_b[ql + 1] - a0;
    if (n == 0 || n > (uint32_t)kBoundCap) return;  // longer lists take another grouping
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) s_r[i] = b[a0 + i];
    lds_bitonic(s_r, s_ix, n, BoundLess());
    const int lane = threadIdx.x & 63;
    const uint32_t npairs = n / 2;
    for (uint32_t base = 0; base < npairs; base += blockDim.x) {
        const uint32_t i = base + threadIdx.x;
        bool keep = false;
        Cand c{0, 0, 0, 0, 0};
        if (i < npairs) {
            const Bound x = s_r[s_ix[2 * i]], y = s_r[s_ix[2 * i + 1]];
            c = Cand{ql, x.s, x.d, x.qpos, y.qpos + k};
            keep = c.qe - c.qs >= M;
        }
        const uint64_t mk = __ballot(keep);
        if (mk) {
            const int leader = __ffsll((unsigned long long)mk) - 1;
            uint32_t at0 = 0;
            if (lane == leader) at0 = atomicAdd(ccount, (uint32_t)__popcll(mk));
            at0 = __shfl(at0, leader, 64);
            if (keep) {
                const uint32_t at = at0 + (uint32_t)__popcll(mk & ((1ull << lane) - 1ull));
                if (at < ccap) cands[at] = c;
                atomicAdd(&cand_per_q[ql], 1u);
            }
        }
    }
}

void launch_pair_bounds(const Bound *b, const uint32_t *qoff_b, int32_t nq, int32_t k,
                        int32_t min_len, Cand *cands, uint32_t ccap, uint32_t *ccount,
                        uint32_t *cand_per_q, hipStream_t st)
{
    if (nq > 0)
        k_pair_bounds<<<nq, kBlock, 0, st>>>(b, qoff_b, k, min_len, cands, ccap, ccount, cand_per_q);
}

// Runs appended in any order go to their query's range (a counting sort by query).
__global__ void k_group_by_query(const Cand *__restrict__ in, uint32_t n,
                                 const uint32_t *__restrict__ qoff_c, uint32_t *__restrict__ cur,
                                 Cand *__restrict__ out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Cand c = in[i];
    out[qoff_c[c.q] + atomicAdd(&cur[c.q], 1u)] = c;
}

void launch_group_by_query(const Cand *in, uint32_t n, const uint32_t *qoff_c, uint32_t *cur,
                           Cand *out, hipStream_t st)
{
    if (n) k_group_by_query<<<(n + kBlock - 1) / kBlock, kBlock, 0, st>>>(in, n, qoff_c, cur, out);
}

// ------------------------------------------------------------------ S4: radix sort
// Stable LSD radix sort, 8 bits per pass: digit histogram per tile, one scan of the
// digit-major histogram matrix, then a stable scatter.  In the scatter, each wave
// ranks its keys with ballot-built peer masks (lanes holding the same digit) and
// per-wave digit counters in LDS; the tile is then reordered in LDS so that the
// global writes of each digit run are contiguous.
// The keys and count slots of one radix tile: its key range [base, base + cnt) and
// count index hidx + digit * stride.  Plain tiles split [0, n) evenly and keep
// digit-major counts over nb tiles; segmented tiles come from a table (tiles of
// a graph's capacity past the wave count zero keys after every real tile).
struct TileView {
    uint32_t base, cnt, hidx, stride;
};

__device__ __forceinline__ TileView tile_view(uint32_t tile, uint32_t n, uint32_t nb,
                                              const SortTile *__restrict__ tiles, uint32_t ntile)
{
    TileView v;
    if (tiles) {
        if (tile < ntile) {
            const SortTile t = tiles[tile];
            v = TileView{t.start, t.count, t.hbase + t.tq, t.nt};
        } else {
            v = TileView{0, 0, tile * (uint32_t)kRadix, 1};
        }
    } else {
        v.base = tile * (uint32_t)kSortTile;
        v.cnt = v.base < n ? min((uint32_t)kSortTile, n - v.base) : 0u;
        v.hidx = tile;
        v.stride = nb;
    }
    return v;
}

// Blocks are handed to the 8 XCDs in turn (block b to XCD b % 8), and each XCD
// has its own L2.  Consecutive tiles write neighbouring runs of each digit, which
// share cache lines at their ends; giving every XCD one contiguous chunk of the
// active tiles (in block order within the chunk) keeps those shared lines in one
// L2, where the partial writes merge instead of each L2 reading the line back from
// HBM.  A bijection on [0, active); blocks past it keep their own number.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t active)
{
    if (b >= active) return b;
    const uint32_t x = b & 7u, slot = b >> 3, q = active >> 3, r = active & 7u;
    return x * q + min(x, r) + slot;
}

constexpr int kHistCopies = 16;

__global__ __launch_bounds__(kBlock) void k_rs_hist(const uint64_t *__restrict__ keys, uint32_t n,
                                                    int shift, uint32_t *__restrict__ hist,
                                                    uint32_t nb, const WaveCtl *__restrict__ ctl,
                                                    const SortTile *__restrict__ tiles)
{
    __shared__ uint32_t h[kHistCopies * (kRadix + 1)];
    uint32_t ntile = nb;
    if (ctl) {  // shift holds the pass number; tiles past the wave's keys count zeros
        n = ctl->H;
        shift = ctl->lay.bp + kRadixBits * shift;
        if (tiles) {
            tiles += ctl->tile0;
            ntile = ctl->ntile;
        }
    }
    const uint32_t active = tiles ? ntile : (n + kSortTile - 1) / kSortTile;
    const TileView tv = tile_view(xcd_tile(blockIdx.x, active), n, nb, tiles, ntile);
    // kHistCopies counters per digit (lane l adds to copy l % kHistCopies, copies
    // kRadix + 1 words apart so that they sit in different banks): keys of one digit
    // are common in a tile (repeats, and the digits above the ones already sorted),
    // and lanes adding to one address take turns
#pragma unroll
    for (int c = 0; c < kHistCopies; ++c) h[c * (kRadix + 1) + threadIdx.x] = 0;
    // keys read two per 16-byte load (tile starts are only 8-byte aligned)
    u64x2_a8 k[kSortItems / 2];
#pragma unroll
    for (int r = 0; r < kSortItems / 2; ++r) {
        const uint32_t i = 2 * (r * kBlock + threadIdx.x);
        if (i + 1 < tv.cnt) k[r] = *reinterpret_cast<const u64x2_a8 *>(keys + tv.base + i);
        else if (i < tv.cnt) k[r].x = keys[tv.base + i];
    }
    __syncthreads();
    uint32_t *mine = h + (threadIdx.x % kHistCopies) * (kRadix + 1);
#pragma unroll
    for (int r = 0; r < kSortItems / 2; ++r) {
        const uint32_t i = 2 * (r * kBlock + threadIdx.x);
        if (i < tv.cnt) atomicAdd(&mine[(uint32_t)(k[r].x >> shift) & (kRadix - 1)], 1u);
        if (i + 1 < tv.cnt) atomicAdd(&mine[(uint32_t)(k[r].y >> shift) & (kRadix - 1)], 1u);
    }
    __syncthreads();
    uint32_t tot = 0;
#pragma unroll
    for (int c = 0; c < kHistCopies; ++c) tot += h[c * (kRadix + 1) + threadIdx.x];
    hist[(size_t)tv.hidx + (size_t)threadIdx.x * tv.stride] = tot;
}

// One-sweep passes (no per-pass histogram kernel): a tile learns how many keys of
// each digit the tiles before it hold by decoupled look-back over per-tile
// descriptors [tag | flag | count] (tag = pass + 1, flag 1 = this tile's count,
// 2 = count of every tile up to this one).  Tiles are numbered in start order by
// a counter, so every tile waited on has started and publishes its own count
// before it waits; each wait is still bounded, and running out sets *fail (the
// pass's output is then invalid and the caller sorts again without look-back).
struct Lookback {
    unsigned long long *desc;  // [tiles][kRadix]
    const uint32_t *base;      // [kRadix] keys of smaller digits in the whole input
    uint32_t *counter;         // next tile number of this pass
    uint32_t *fail;
    uint32_t tag;
};

constexpr int kDescFlagShift = 58;
constexpr int kDescTagShift = 60;
constexpr unsigned long long kDescCount = (1ull << kDescFlagShift) - 1;
constexpr uint32_t kSpinLimit = 1u << 20;

__device__ __forceinline__ void desc_store(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long desc_load(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Keys of digit d in tiles before `tile` (thread d of the block; cnt = this tile's).
__device__ uint32_t look_back(const Lookback &lb, uint32_t tile, uint32_t d, uint32_t cnt)
{
    unsigned long long *me = lb.desc + (size_t)tile * kRadix + d;
    const unsigned long long tag = (unsigned long long)lb.tag << kDescTagShift;
    if (tile == 0) {
        desc_store(me, tag | (2ull << kDescFlagShift) | cnt);
        return 0;
    }
    desc_store(me, tag | (1ull << kDescFlagShift) | cnt);
    unsigned long long excl = 0;
    int64_t j = (int64_t)tile - 1;
    uint32_t spins = 0;
    while (j >= 0) {
        const unsigned long long w = desc_load(lb.desc + (size_t)j * kRadix + d);
        const uint32_t flag = (uint32_t)(w >> kDescFlagShift) & 3u;
        if ((uint32_t)(w >> kDescTagShift) != lb.tag || flag == 0) {
            if (++spins > kSpinLimit) {
                atomicOr(lb.fail, 1u);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        excl += w & kDescCount;
        if (flag == 2) break;
        --j;
    }
    desc_store(me, tag | (2ull << kDescFlagShift) | (excl + cnt));
    return (uint32_t)excl;
}

// Key-only passes: eight waves per SIMD (64 VGPRs) and under 20 KiB of LDS let
// eight tiles share a CU, so more loads and stores are in flight while tiles rank.
template <bool VALS, bool LB>
__global__ __launch_bounds__(kBlock, (VALS || LB) ? 4 : 8) void k_rs_scatter(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint64_t *__restrict__ kout,
    uint32_t *__restrict__ vout, uint32_t n, int shift, const uint32_t *__restrict__ hist,
    uint32_t nb, Lookback lb, const WaveCtl *__restrict__ ctl, const SortTile *__restrict__ tiles)
{
    uint32_t ntile = nb;
    if (ctl) {  // shift holds the pass number
        n = ctl->H;
        shift = ctl->lay.bp + kRadixBits * shift;
        if (tiles) {
            tiles += ctl->tile0;
            ntile = ctl->ntile;
        }
    }
    __shared__ uint64_t s_k[kSortTile];
    __shared__ uint32_t s_v[VALS ? kSortTile : 1];
    __shared__ uint16_t s_wc[kBlock / 64][kRadix];  // per-wave digit counts, then positions
    __shared__ uint32_t s_off[kRadix];  // output position of digit d's keys minus their tile position
    __shared__ uint32_t s_tile;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) s_wc[i][threadIdx.x] = 0;
    if (LB && threadIdx.x == 0) s_tile = atomicAdd(lb.counter, 1u);
    __syncthreads();
    const uint32_t tile =
        LB ? s_tile : xcd_tile(blockIdx.x, tiles ? ntile : (n + kSortTile - 1) / kSortTile);
    const TileView tv = tile_view(tile, n, nb, tiles, ntile);
    if (tv.cnt == 0) return;  // whole block: only capacity tiles of a graph are empty
    const uint32_t sub = w * 64 * kSortItems;  // this wave's first key in the tile
    const uint64_t below = (1ull << lane) - 1ull;
    uint64_t k[kSortItems];
    uint32_t v[kSortItems], rank[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const uint32_t idx = sub + r * 64 + lane;
        const bool ok = idx < tv.cnt;
        k[r] = ok ? kin[tv.base + idx] : 0ull;
        if (VALS) v[r] = ok ? vin[tv.base + idx] : 0u;
        const uint32_t d = (uint32_t)(k[r] >> shift) & (kRadix - 1);
        uint64_t peers = __ballot(ok);
        // lanes past the tile hold key 0 (digit 0), so they are clear in every
        // bit's ballot, and peers never holds them
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            const int32_t mk = (int32_t)(d << (31 - b)) >> 31;  // all ones when bit b is set
            const uint64_t bb = __ballot(mk != 0);
            peers &= ~(bb ^ (((uint64_t)(uint32_t)mk << 32) | (uint32_t)mk));
        }
        const uint32_t before = s_wc[w][d];
        rank[r] = before + (uint32_t)__popcll(peers & below);
        __builtin_amdgcn_wave_barrier();
        if (ok && (peers & below) == 0) s_wc[w][d] = (uint16_t)(before + (uint32_t)__popcll(peers));
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    {
        const uint32_t d = threadIdx.x;
        uint32_t run = 0, wc[kBlock / 64];
#pragma unroll
        for (int i = 0; i < kBlock / 64; ++i) {
            wc[i] = run;
            run += s_wc[i][d];
        }
        uint32_t tot;
        const uint32_t start = block_excl_scan<uint32_t>(run, &tot);  // digit d's first key in the tile
#pragma unroll
        for (int i = 0; i < kBlock / 64; ++i) s_wc[i][d] = (uint16_t)(start + wc[i]);
        const uint32_t gbase = LB ? lb.base[d] + look_back(lb, tile, d, run)
                                  : hist[(size_t)tv.hidx + (size_t)d * tv.stride];
        s_off[d] = gbase - start;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const uint32_t idx = sub + r * 64 + lane;
        if (idx < tv.cnt) {
            const uint32_t d = (uint32_t)(k[r] >> shift) & (kRadix - 1);
            const uint32_t pos = (uint32_t)s_wc[w][d] + rank[r];
            s_k[pos] = k[r];
            if (VALS) s_v[pos] = v[r];
        }
    }
    __syncthreads();
    const uint32_t tn = tv.cnt;
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const uint32_t i = r * kBlock + threadIdx.x;
        if (i < tn) {
            const uint64_t key = s_k[i];
            const uint32_t d = (uint32_t)(key >> shift) & (kRadix - 1);
            const uint32_t o = s_off[d] + i;
            kout[o] = key;
            if (VALS) vout[o] = s_v[i];
        }
    }
}

// Digit counts of every pass in one read of the keys: hist[p][d] = keys whose
// digit p (bits lo + 8p .. lo + 8p + 7) is d.
__global__ __launch_bounds__(kBlock) void k_os_hist(const uint64_t *__restrict__ keys, uint32_t n,
                                                    int lo, int passes,
                                                    uint32_t *__restrict__ hist)
{
    __shared__ uint32_t h[8][kRadix];
    for (int p = 0; p < passes; ++p) h[p][threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const uint64_t key = keys[i];
        for (int p = 0; p < passes; ++p)
            atomicAdd(&h[p][(uint32_t)(key >> (lo + 8 * p)) & (kRadix - 1)], 1u);
    }
    __syncthreads();
    for (int p = 0; p < passes; ++p) {
        const uint32_t c = h[p][threadIdx.x];
        if (c) atomicAdd(&hist[p * kRadix + threadIdx.x], c);
    }
}

// hist[p][d] -> keys of digits below d in pass p (one block).
__global__ __launch_bounds__(kBlock) void k_os_scan(uint32_t *__restrict__ hist, int passes)
{
    for (int p = 0; p < passes; ++p) {
        uint32_t tot;
        const uint32_t e = block_excl_scan<uint32_t>(hist[p * kRadix + threadIdx.x], &tot);
        hist[p * kRadix + threadIdx.x] = e;
    }
}

// Last node of a replayed wave graph: move the cursor to the next planned wave
// (the first node, the wave preparation, takes the plan entry at the cursor).
__global__ void k_wave_end(uint32_t *__restrict__ cursor) { *cursor += 1; }

void launch_wave_end(uint32_t *cursor, hipStream_t st) { k_wave_end<<<1, 1, 0, st>>>(cursor); }

__global__ void k_fill_u32(uint32_t *__restrict__ p, size_t n, uint32_t v)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

void launch_fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t st)
{
    if (n == 0) return;
    const size_t nb = std::min<size_t>((n + kBlock - 1) / kBlock, 4096);
    k_fill_u32<<<(uint32_t)nb, kBlock, 0, st>>>(p, n, v);
}

// Streaming read of `bytes` bytes (a multiple of 16) for memory-counter
// calibration: every 16-byte vector is loaded once, coalesced, and folded into a
// per-thread sum; each block adds its sum to *sum with one atomic, so the kernel
// writes 8 bytes per block and reads exactly the buffer.
__global__ void k_stream_read(const uint4 *__restrict__ src, size_t n16,
                              unsigned long long *__restrict__ sum)
{
    __shared__ unsigned long long part[kBlock / 64];
    unsigned long long acc = 0;
    const size_t step = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += step) {
        const uint4 v = src[i];
        acc += (unsigned long long)v.x + v.y + v.z + v.w;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kBlock / 64; ++w) t += part[w];
        atomicAdd(sum, t);
    }
}

void launch_stream_read(const void *src, size_t bytes, unsigned long long *sum, hipStream_t st)
{
    const size_t n16 = bytes / 16;
    if (n16 == 0) return;
    const size_t nb = std::min<size_t>((n16 + kBlock - 1) / kBlock, 8192);
    k_stream_read<<<(uint32_t)nb, kBlock, 0, st>>>(static_cast<const uint4 *>(src), n16, sum);
}

// Two arrays set to v in one launch (a graph node less than two fills).
__global__ void k_fill2_u32(uint32_t *__restrict__ a, size_t na, uint32_t *__restrict__ b,
                            size_t nb, uint32_t v)
{
    const size_t step = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < na + nb; i += step) {
        if (i < na) a[i] = v;
        else b[i - na] = v;
    }
}

void launch_fill2_u32(uint32_t *a, size_t na, uint32_t *b, size_t nb, uint32_t v, hipStream_t st)
{
    if (na + nb == 0) return;
    const size_t blocks = std::min<size_t>((na + nb + kBlock - 1) / kBlock, 4096);
    k_fill2_u32<<<(uint32_t)blocks, kBlock, 0, st>>>(a, na, b, nb, v);
}

// Scratch of a one-sweep sort of n keys: digit counts (8 passes x 256), tile
// counters and the failure flag, then the descriptors.
constexpr size_t kOsHead = (8 * kRadix + 64) * sizeof(uint32_t);

size_t onesweep_scratch_bytes(uint32_t n)
{
    const size_t nt = (n + kSortTile - 1) / kSortTile;
    return kOsHead + nt * kRadix * sizeof(unsigned long long);
}

void onesweep_prepare(const uint64_t *keys, uint32_t n, int lo, int hi, void *scratch,
                      hipStream_t st)
{
    if (n == 0 || hi <= lo) return;
    const int passes = (hi - lo + kRadixBits - 1) / kRadixBits;
    uint32_t *hist = static_cast<uint32_t *>(scratch);
    launch_fill_u32(hist, onesweep_scratch_bytes(n) / 4, 0u, st);
    const uint32_t hb = std::min<uint32_t>((n + kBlock * 8 - 1) / (kBlock * 8), 4096);
    k_os_hist<<<hb, kBlock, 0, st>>>(keys, n, lo, passes, hist);
    k_os_scan<<<1, kBlock, 0, st>>>(hist, passes);
}

void onesweep_pass(const uint64_t *kin, uint64_t *kout, uint32_t n, int lo, int pass,
                   void *scratch, hipStream_t st)
{
    if (n == 0) return;
    uint32_t *hist = static_cast<uint32_t *>(scratch);
    uint32_t *counters = hist + 8 * kRadix;  // [8], then the failure flag at [8]
    auto *desc = reinterpret_cast<unsigned long long *>(static_cast<char *>(scratch) + kOsHead);
    const uint32_t nt = (n + kSortTile - 1) / kSortTile;
    const Lookback lb{desc, hist + pass * kRadix, counters + pass, counters + 8,
                      (uint32_t)pass + 1};
    k_rs_scatter<false, true><<<nt, kBlock, 0, st>>>(kin, nullptr, kout, nullptr, n,
                                                     lo + kRadixBits * pass, nullptr, nt, lb,
                                                     nullptr, nullptr);
}

const uint32_t *onesweep_fail_flag(const void *scratch)
{
    return static_cast<const uint32_t *>(scratch) + 8 * kRadix + 8;
}

size_t radix_hist_needed(uint32_t n)
{
    const size_t nb = (n + kSortTile - 1) / kSortTile;
    return nb * kRadix + 1;
}

void launch_rs_hist(const uint64_t *keys, uint32_t n, int shift, uint32_t *hist, hipStream_t st)
{
    const uint32_t nb = (n + kSortTile - 1) / kSortTile;
    k_rs_hist<<<nb, kBlock, 0, st>>>(keys, n, shift, hist, nb, nullptr, nullptr);
}

void launch_rs_scan(uint32_t *hist, uint32_t n, uint32_t *partials, hipStream_t st)
{
    const uint32_t nb = (n + kSortTile - 1) / kSortTile;
    scan_impl<uint32_t, uint32_t>(hist, hist, (int64_t)nb * kRadix, partials, st);
}

void launch_rs_scatter(const uint64_t *kin, const uint32_t *vin, uint64_t *kout, uint32_t *vout,
                       uint32_t n, int shift, const uint32_t *hist, hipStream_t st)
{
    const uint32_t nb = (n + kSortTile - 1) / kSortTile;
    const Lookback none{};
    if (vin)
        k_rs_scatter<true, false><<<nb, kBlock, 0, st>>>(kin, vin, kout, vout, n, shift, hist, nb,
                                                         none, nullptr, nullptr);
    else
        k_rs_scatter<false, false><<<nb, kBlock, 0, st>>>(kin, nullptr, kout, nullptr, n, shift,
                                                          hist, nb, none, nullptr, nullptr);
}

// One radix pass within query segments, in three launches: digit counts per tile
// of the table (in its segmented layout), their exclusive scan (ntile * 256
// counts), the stable scatter.
void launch_rs_hist_seg(const uint64_t *kin, uint32_t ntile, int shift, const SortTile *tiles,
                        uint32_t *hist, hipStream_t st)
{
    if (ntile) k_rs_hist<<<ntile, kBlock, 0, st>>>(kin, 0, shift, hist, ntile, nullptr, tiles);
}

void launch_rs_scan_seg(uint32_t *hist, uint32_t ntile, uint32_t *partials, hipStream_t st)
{
    if (ntile) scan_impl<uint32_t, uint32_t>(hist, hist, (int64_t)ntile * kRadix, partials, st);
}

void launch_rs_scatter_seg(const uint64_t *kin, uint64_t *kout, uint32_t ntile, int shift,
                           const SortTile *tiles, const uint32_t *hist, hipStream_t st)
{
    const Lookback none{};
    if (ntile)
        k_rs_scatter<false, false><<<ntile, kBlock, 0, st>>>(kin, nullptr, kout, nullptr, 0, shift,
                                                             hist, ntile, none, nullptr, tiles);
}

// The same pass for a graph-replayed wave: the wave's tiles (ctl->tile0,
// ctl->ntile) and shift (digit `pass` above the qpos bits) are read on the device;
// the grid and count layout cover ntile_cap tiles.
void launch_rs_pass_ctl(const uint64_t *kin, uint64_t *kout, uint32_t ntile_cap, int pass,
                        const SortTile *tiles, uint32_t *hist, uint32_t *partials,
                        const WaveCtl *ctl, hipStream_t st)
{
    const uint32_t nb = std::max<uint32_t>(1, ntile_cap);
    k_rs_hist<<<nb, kBlock, 0, st>>>(kin, 0, pass, hist, nb, ctl, tiles);
    scan_impl<uint32_t, uint32_t>(hist, hist, (int64_t)nb * kRadix, partials, st);
    const Lookback none{};
    k_rs_scatter<false, false><<<nb, kBlock, 0, st>>>(kin, nullptr, kout, nullptr, 0, pass, hist,
                                                      nb, none, ctl, tiles);
}

int radix_sort(uint64_t *keys, uint64_t *keys_alt, uint32_t *vals, uint32_t *vals_alt,
               uint32_t n, int lo, int hi, uint32_t *hist, uint32_t *partials, hipStream_t st)
{
    int cur = 0;
    if (n <= 1 || hi <= lo) return 0;
    for (int shift = lo; shift < hi; shift += kRadixBits) {
        uint64_t *kin = cur ? keys_alt : keys, *kout = cur ? keys : keys_alt;
        uint32_t *vin = cur ? vals_alt : vals, *vout = cur ? vals : vals_alt;
        launch_rs_hist(kin, n, shift, hist, st);
        launch_rs_scan(hist, n, partials, st);
        launch_rs_scatter(kin, vals ? vin : nullptr, kout, vout, n, shift, hist, st);
        cur ^= 1;
    }
    return cur;
}

// ------------------------------------------------------------------ S4: drop lone diagonals
// A run of one hit covers [qpos, qpos + span), so when M > span (Section 2.2's
// minimum HSP length above the seed span) only hits whose (q, s, diag) group holds
// another hit can end up in a kept run.  At the bank's scale nearly every hit is
// alone on its diagonal, so each query's hits are filtered before grouping: one
// block per query counts the groups in two bit tables (seen once, seen again) in
// LDS, indexed by a hash of (s, diag), and keeps only hits whose slot was seen
// again.  Every member of a real group shares its slot, so no group loses a hit;
// a lone hit whose slot it shares with another group is kept too and forms a run
// too short to keep.  Further rounds with another hash run over what is left
// while they still drop keys.  The kept keys, in qpos order, are then sorted by the
// whole key in LDS (keys are distinct: a query window meets a posting once), the
// order the stable radix sort on (s, diag) gives.  Queries whose kept hits exceed
// the LDS sort are left in qpos order and flagged.
constexpr int kFiltBits = 18;                          // slots per bit table: 2^18
constexpr uint32_t kFiltWords = 1u << (kFiltBits - 5);  // 32-bit words per table
constexpr uint32_t kFiltCap = 2 * kFiltWords * 4 / 8;  // keys the tables' LDS holds (8192)
constexpr uint32_t kFiltSmall = 512;                   // fewer keys are sorted unfiltered
constexpr uint32_t kFiltMax = 2u << kFiltBits;         // more keys would fill the tables
constexpr uint32_t kFiltRounds = 6;

// Slot of a (q, s, diag) group in round r: the group bits folded to 32 and mixed
// with the 32-bit finalizer of MurmurHash3 (Appleby), seeded by the round.  Groups
// that fold alike share a slot in every round; that only keeps a few lone hits.
__device__ __forceinline__ uint32_t diag_slot(uint64_t grp, uint32_t round)
{
    uint32_t x = (uint32_t)grp ^ ((uint32_t)(grp >> 32) * 0x85EBCA6Bu) ^ (round * 0x9E3779B9u);
    x ^= x >> 16;
    x *= 0x85EBCA6Bu;
    x ^= x >> 13;
    x *= 0xC2B2AE35u;
    x ^= x >> 16;
    return x >> (32 - kFiltBits);
}

constexpr int kFiltBlock = 1024;  // threads of a filter block
constexpr int kFiltItems = 8;     // keys per thread and batch, kFiltBlock apart
constexpr uint32_t kFiltBatch = kFiltBlock * kFiltItems;
constexpr int kFiltWaves = kFiltBlock / 64;

// The filter block's LDS: the two bit tables, later the kept keys; kept keys per
// slab and wave and their exclusive scan.
struct FiltLds {
    uint64_t buf[kFiltCap];
    uint32_t cnt[kFiltItems * kFiltWaves];
    uint32_t pre[kFiltItems * kFiltWaves];
    uint32_t tot;
};

// Stable compaction of one batch: keys v[j] (input index base + j * kFiltBlock +
// thread) with keep[j] set go to dst + out, in input order, placed by ballots per
// slab and wave and one scan of those counts.  Returns the batch's kept count.
__device__ __forceinline__ uint32_t keep_batch(const uint64_t (&v)[kFiltItems],
                                               const bool (&keep)[kFiltItems],
                                               uint64_t *__restrict__ dst, uint32_t out,
                                               FiltLds &L)
{
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    const uint64_t below = (1ull << lane) - 1ull;
    uint64_t mask[kFiltItems];
#pragma unroll
    for (int j = 0; j < kFiltItems; ++j) {
        mask[j] = __ballot(keep[j]);
        if (lane == 0) L.cnt[j * kFiltWaves + w] = (uint32_t)__popcll(mask[j]);
    }
    __syncthreads();
    if (w == 0) {  // slab-major, wave-minor exclusive scan of the counts
        constexpr int kPer = kFiltItems * kFiltWaves / 64;  // counts per lane
        static_assert(kPer * 64 == kFiltItems * kFiltWaves, "whole counts per lane");
        uint32_t c[kPer], x = 0;
#pragma unroll
        for (int e = 0; e < kPer; ++e) {
            c[e] = L.cnt[kPer * lane + e];
            x += c[e];
        }
        const uint32_t mine = x;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, 64);
            if ((int)lane >= o) x += y;
        }
        uint32_t run = x - mine;
#pragma unroll
        for (int e = 0; e < kPer; ++e) {
            L.pre[kPer * lane + e] = run;
            run += c[e];
        }
        if (lane == 63) L.tot = x;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kFiltItems; ++j)
        if ((mask[j] >> lane) & 1ull)
            dst[out + L.pre[j * kFiltWaves + w] + (uint32_t)__popcll(mask[j] & below)] = v[j];
    // the next batch rewrites cnt only before its first barrier, which every wave
    // reaches after reading pre and tot here
    return L.tot;
}

// Marks slot diag_slot(key >> bp, round) of each valid key in the tables: seen
// once, seen again.
__device__ __forceinline__ void mark_batch(const uint64_t (&v)[kFiltItems],
                                           const bool (&valid)[kFiltItems], int bp,
                                           uint32_t round, uint32_t *__restrict__ seen,
                                           uint32_t *__restrict__ again)
{
#pragma unroll
    for (int j = 0; j < kFiltItems; ++j) {
        if (valid[j]) {
            const uint32_t h = diag_slot(v[j] >> bp, round), bit = 1u << (h & 31u);
            if (atomicOr(&seen[h >> 5], bit) & bit) atomicOr(&again[h >> 5], bit);
        }
    }
}

__device__ __forceinline__ bool slot_again(uint64_t key, int bp, uint32_t round,
                                           const uint32_t *__restrict__ again)
{
    const uint32_t h = diag_slot(key >> bp, round);
    return (again[h >> 5] >> (h & 31u)) & 1u;
}

// Filter rounds `round`, round + 1, ... over the m keys at k, in place; each
// round's compaction reads a batch before any of its keys move, and keys only
// move down.  The rounds stop once one drops fewer than an eighth of the keys
// (the rest are nearly all real groups).  Returns the kept count.
__device__ __forceinline__ uint32_t filter_rounds(uint64_t *__restrict__ k, uint32_t m, uint32_t round, int bp,
                                  FiltLds &L)
{
    uint32_t *seen = reinterpret_cast<uint32_t *>(L.buf), *again = seen + kFiltWords;
    for (; round < kFiltRounds && m >= kFiltSmall && m <= kFiltMax; ++round) {
        for (uint32_t i = threadIdx.x; i < 2 * kFiltWords; i += kFiltBlock) seen[i] = 0u;
        __syncthreads();
        for (uint32_t base = 0; base < m; base += kFiltBatch) {
            uint64_t v[kFiltItems];
            bool in[kFiltItems];
#pragma unroll
            for (int j = 0; j < kFiltItems; ++j) {
                const uint32_t i = base + j * kFiltBlock + threadIdx.x;
                in[j] = i < m;
                v[j] = in[j] ? k[i] : 0ull;
            }
            mark_batch(v, in, bp, round, seen, again);
        }
        __syncthreads();
        uint32_t out = 0;
        for (uint32_t base = 0; base < m; base += kFiltBatch) {
            uint64_t v[kFiltItems];
            bool keep[kFiltItems];
#pragma unroll
            for (int j = 0; j < kFiltItems; ++j) {
                const uint32_t i = base + j * kFiltBlock + threadIdx.x;
                v[j] = i < m ? k[i] : 0ull;
            }
#pragma unroll
            for (int j = 0; j < kFiltItems; ++j)
                keep[j] = base + j * kFiltBlock + threadIdx.x < m && slot_again(v[j], bp, round, again);
            out += keep_batch(v, keep, k, out, L);
        }
        __syncthreads();
        const uint32_t before = m;
        m = out;
        if ((before - m) * 8u < before) break;
    }
    return m;
}

// The m kept keys of wave query ql at k: sorted by the whole key in LDS (keys are
// distinct: a query window meets a posting once), the order the stable radix sort
// on (s, diag) gives.  A query over the LDS sort is left in qpos order and flagged;
// a replayed wave drops its hits and flags the query for the host path, which
// radix-sorts them after the compaction.
__device__ __forceinline__ void filter_finish(uint64_t *__restrict__ k, uint32_t m, int32_t ql,
                              uint32_t *__restrict__ kept, uint32_t *__restrict__ flag,
                              WaveCtl *__restrict__ ctl, FiltLds &L)
{
    const bool over = m > kFiltCap;
    if (threadIdx.x == 0) {
        kept[ql] = (over && ctl) ? 0u : m;
        if (over) {
            if (ctl) ctl->qflag[ctl->qa + ql] = 1u;
            else atomicOr(flag, 1u);
        }
    }
    if (over) return;
    uint32_t n2 = 1;
    while (n2 < m) n2 <<= 1;
    for (uint32_t i = threadIdx.x; i < n2; i += kFiltBlock) L.buf[i] = i < m ? k[i] : ~0ull;
    __syncthreads();
    for (uint32_t kk = 2; kk <= n2; kk <<= 1) {
        for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < n2; i += kFiltBlock) {
                const uint32_t l = i ^ j;
                if (l > i) {
                    const uint64_t x = L.buf[i], y = L.buf[l];
                    if ((i & kk) == 0 ? y < x : x < y) {
                        L.buf[i] = y;
                        L.buf[l] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t i = threadIdx.x; i < m; i += kFiltBlock) k[i] = L.buf[i];
}

// Wave query `r`-th in the filter's order: blocks take the wave's queries largest
// first, so the longest filters start early (a replayed wave's order array covers
// the batch; a host-run wave's, the wave).
__device__ __forceinline__ int32_t filter_query(const int32_t *__restrict__ order, int32_t qa,
                                                const WaveCtl *ctl)
{
    return !order ? (int32_t)blockIdx.x : order[(ctl ? qa : 0) + (int32_t)blockIdx.x];
}

// Hits of wave query ql: [hrel[qoff[qa + ql] - g0], hrel[qoff[qa + ql + 1] - g0]),
// already gathered as keys.
__global__ __launch_bounds__(kFiltBlock) void k_hit_filter(uint64_t *__restrict__ keys,
                                                           const uint32_t *__restrict__ hrel,
                                                           const int64_t *__restrict__ qoff,
                                                           int32_t qa, int64_t g0, int32_t nqw,
                                                           int bp,
                                                           const int32_t *__restrict__ order,
                                                           uint32_t *__restrict__ kept,
                                                           uint32_t *__restrict__ flag,
                                                           WaveCtl *__restrict__ ctl)
{
    __shared__ FiltLds L;
    if (ctl) {
        qa = ctl->qa;
        g0 = ctl->g0;
        nqw = ctl->nqw;
        bp = ctl->lay.bp;
    }
    if ((int32_t)blockIdx.x >= nqw) {
        if (threadIdx.x == 0) kept[blockIdx.x] = 0;
        return;
    }
    const int32_t ql = filter_query(order, qa, ctl);
    const uint32_t a = hrel[qoff[qa + ql] - g0];
    uint64_t *k = keys + a;
    const uint32_t m = filter_rounds(k, hrel[qoff[qa + ql + 1] - g0] - a, 0, bp, L);
    filter_finish(k, m, ql, kept, flag, ctl, L);
}

// The gather and the first filter round in one pass per query, no key stored
// before it: each block (one query) builds its hits' keys from the postings, marks
// their (s, diag) slots, then writes only the keys whose slot was seen again, at
// the query's place in `keys`; a query of one batch keeps its keys in registers
// between the two steps, a longer one builds them again.  A query with fewer hits
// than kFiltSmall or more than kFiltMax is written whole.
//
// A batch of kFiltBatch consecutive hits covers the positions pa..pb.  Each position
// that starts inside the batch marks its first hit's slot with its index, and a
// forward fill (block max-scan) gives every hit its position; the hit's posting is
// then the position's list start plus its rank in the position.  A query of at most
// kFusePos positions has its hit offsets and list starts staged in LDS, and the
// block finds pa and pb by testing kFiltBlock positions at once.  A longer one has
// every 2^sb-th offset staged: one thread searches pa and pb, and the batch's
// offsets and list starts are read from global memory (or, over more than
// kFusePosBatch positions, each hit searches its own position).
constexpr int32_t kFusePos = 3832;       // positions whose offsets and list starts are staged
constexpr int32_t kFusePosBatch = 3832;  // positions one batch may span for the forward fill

__global__ __launch_bounds__(kFiltBlock) void k_gather_filter(
    const uint32_t *__restrict__ hrel, const uint32_t *__restrict__ pbase,
    const int2 *__restrict__ post, const int64_t *__restrict__ qoff, int32_t qa, int64_t g0,
    int32_t nqw, HitKeyLayout lay, const int32_t *__restrict__ order,
    uint64_t *__restrict__ keys, uint32_t *__restrict__ kept, uint32_t *__restrict__ flag,
    WaveCtl *__restrict__ ctl)
{
    __shared__ FiltLds L;
    __shared__ uint32_t s_h[kFusePos + 1];  // hit offsets (every 2^sb-th position)
    __shared__ uint32_t s_b[kFusePos + 1];  // list starts (sb = 0), or the batch's list start
                                            // minus first hit per position (sb > 0)
    __shared__ uint16_t s_pos[kFiltBatch];  // batch hit -> position - pa
    __shared__ int32_t s_wmax[kFiltWaves];
    __shared__ int32_t s_pab[2];
    static_assert(kFusePosBatch <= kFusePos + 1, "a batch's list starts fit s_b");
    if (ctl) {
        qa = ctl->qa;
        g0 = ctl->g0;
        nqw = ctl->nqw;
        lay = ctl->lay;
    }
    if ((int32_t)blockIdx.x >= nqw) {
        if (threadIdx.x == 0) kept[blockIdx.x] = 0;
        return;
    }
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    const int bp = lay.bp, sh_s = lay.bp + lay.bd, sh_q = lay.bp + lay.bd + lay.bs;
    const int32_t ql = filter_query(order, qa, ctl);
    const uint64_t qpart = sh_q >= 64 ? 0ull : ((uint64_t)(uint32_t)ql << sh_q);
    const int64_t p0 = qoff[qa + ql] - g0;
    const int32_t P = (int32_t)(qoff[qa + ql + 1] - g0 - p0);  // positions of the query
    const uint32_t a = hrel[p0];
    const uint32_t m = hrel[p0 + P] - a;
    uint64_t *k = keys + a;
    int sb = 0;
    while (((P + (1 << sb) - 1) >> sb) > kFusePos) ++sb;
    const int32_t Pc = (P + (1 << sb) - 1) >> sb;  // staged offsets: positions c << sb
    for (int32_t c = threadIdx.x; c < Pc; c += kFiltBlock) {
        s_h[c] = hrel[p0 + ((int64_t)c << sb)] - a;
        if (sb == 0) s_b[c] = pbase[p0 + c];
    }
    if (sb == 0 && threadIdx.x == 0) s_h[P] = m;
    int32_t top = 1;
    while (2 * top < Pc) top <<= 1;
    __syncthreads();
    // position of hit j < m: the last one whose first hit is <= j (positions without
    // hits share their offset with the next one)
    auto locate = [&](uint32_t j) -> int32_t {
        int32_t x = 0;
        for (int32_t s = top; s > 0; s >>= 1) {
            const int32_t t = min(x + s, Pc - 1);
            x = s_h[t] <= j ? t : x;
        }
        x <<= sb;
        for (int32_t s = (1 << sb) >> 1; s > 0; s >>= 1) {
            const int32_t t = min(x + s, P - 1);
            if (hrel[p0 + t] - a <= j) x = t;
        }
        return x;
    };
    auto key_at = [&](int32_t x, const int2 e) -> uint64_t {
        return qpart + ((uint64_t)(uint32_t)(lay.bias - x + e.y) << bp) + (uint64_t)(uint32_t)x +
               ((uint64_t)(uint32_t)e.x << sh_s);
    };
    int32_t pnext = 0;  // no later batch starts before this position
    // keys of hits base + r * kFiltBlock + thread (an index past m stands for hit m - 1)
    auto build = [&](uint32_t base, uint64_t (&v)[kFiltItems]) {
        const uint32_t nb = min((uint32_t)kFiltBatch, m - base), last = base + nb - 1;
        __syncthreads();  // the previous batch is done with s_pos, s_b and s_pab
        if (sb == 0) {
            if (threadIdx.x == 0) s_pab[0] = s_pab[1] = pnext;
            __syncthreads();
            for (int32_t x0 = pnext;; x0 += kFiltBlock) {  // block-uniform
                const int32_t x = x0 + (int32_t)threadIdx.x;
                if (x < P) {
                    const uint32_t f = s_h[x];
                    if (f <= base) atomicMax(&s_pab[0], x);
                    if (f <= last) atomicMax(&s_pab[1], x);
                }
                __syncthreads();
                if (s_pab[1] < x0 + kFiltBlock - 1 || x0 + kFiltBlock >= P) break;
            }
        } else if (threadIdx.x == 0) {
            s_pab[0] = locate(base);
            s_pab[1] = locate(last);
        }
        __syncthreads();
        const int32_t pa = s_pab[0], pb = s_pab[1];
        pnext = pb;
        if (sb == 0 || pb - pa < kFusePosBatch) {
            for (uint32_t i = threadIdx.x; i < nb; i += kFiltBlock) s_pos[i] = 0;
            __syncthreads();
            for (int32_t x = pa + (int32_t)threadIdx.x; x <= pb; x += kFiltBlock) {
                uint32_t f, n;
                if (sb == 0) {
                    f = s_h[x];
                    n = s_h[x + 1] - f;
                } else {
                    f = hrel[p0 + x] - a;
                    n = hrel[p0 + x + 1] - a - f;
                    s_b[x - pa] = pbase[p0 + x] - f;
                }
                if (n > 0 && f > base) s_pos[f - base] = (uint16_t)(x - pa);
            }
            __syncthreads();
            // forward fill: a block max-scan, kFiltItems consecutive hits per thread
            int32_t run[kFiltItems], mx = 0;
#pragma unroll
            for (int e = 0; e < kFiltItems; ++e) {
                const uint32_t i = threadIdx.x * kFiltItems + e;
                mx = max(mx, i < nb ? (int32_t)s_pos[i] : 0);
                run[e] = mx;
            }
            int32_t x = mx;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int32_t y = __shfl_up(x, o, 64);
                if ((int)lane >= o) x = max(x, y);
            }
            if (lane == 63) s_wmax[w] = x;
            int32_t ex = __shfl_up(x, 1, 64);
            __syncthreads();
            if (lane == 0) ex = 0;
            for (uint32_t i = 0; i < w; ++i) ex = max(ex, s_wmax[i]);
#pragma unroll
            for (int e = 0; e < kFiltItems; ++e) {
                const uint32_t i = threadIdx.x * kFiltItems + e;
                if (i < nb) s_pos[i] = (uint16_t)max(ex, run[e]);
            }
            __syncthreads();
            uint32_t jj[kFiltItems], idx[kFiltItems];
            int32_t xs[kFiltItems];
#pragma unroll
            for (int r = 0; r < kFiltItems; ++r) {
                jj[r] = min(base + r * kFiltBlock + threadIdx.x, m - 1);
                const int32_t rel = s_pos[jj[r] - base];
                xs[r] = pa + rel;
                idx[r] = sb == 0 ? s_b[xs[r]] + (jj[r] - s_h[xs[r]]) : jj[r] + s_b[rel];
            }
#pragma unroll
            for (int r = 0; r < kFiltItems; ++r) v[r] = key_at(xs[r], post[idx[r]]);
        } else {
#pragma unroll
            for (int r = 0; r < kFiltItems; ++r) {
                const uint32_t j = min(base + r * kFiltBlock + threadIdx.x, m - 1);
                const int32_t x = locate(j);
                v[r] = key_at(x, post[pbase[p0 + x] + (j - (hrel[p0 + x] - a))]);
            }
        }
    };
    const bool filter = m >= kFiltSmall && m <= kFiltMax;
    uint32_t *seen = reinterpret_cast<uint32_t *>(L.buf), *again = seen + kFiltWords;
    uint64_t v[kFiltItems];
    bool in[kFiltItems];
    if (filter) {
        for (uint32_t i = threadIdx.x; i < 2 * kFiltWords; i += kFiltBlock) seen[i] = 0u;
        for (uint32_t base = 0; base < m; base += kFiltBatch) {
            build(base, v);
#pragma unroll
            for (int r = 0; r < kFiltItems; ++r) in[r] = base + r * kFiltBlock + threadIdx.x < m;
            mark_batch(v, in, bp, 0, seen, again);
        }
        __syncthreads();
        pnext = 0;
    }
    uint32_t out = 0;
    for (uint32_t base = 0; base < m; base += kFiltBatch) {
        if (!filter || m > kFiltBatch) build(base, v);  // one batch: the keys are still here
        bool keep[kFiltItems];
#pragma unroll
        for (int r = 0; r < kFiltItems; ++r) {
            keep[r] = base + r * kFiltBlock + threadIdx.x < m;
            if (filter) keep[r] = keep[r] && slot_again(v[r], bp, 0, again);
        }
        out += keep_batch(v, keep, k, out, L);
    }
    __syncthreads();
    uint32_t n = out;
    if (filter && (m - n) * 8u >= m) n = filter_rounds(k, n, 1, bp, L);
    filter_finish(k, n, ql, kept, flag, ctl, L);
}

// Sum of v[0..n) over the block (kBlock threads); every thread gets it.
__device__ __forceinline__ uint32_t block_sum(const uint32_t *__restrict__ v, uint32_t n)
{
    uint32_t x = 0;
    for (uint32_t i = threadIdx.x; i < n; i += kBlock) x += v[i];
    uint32_t tot;
    block_excl_scan<uint32_t>(x, &tot);
    return tot;
}

// Each query's kept keys to koff[ql] of `out`, after the scan of the kept counts;
// a replayed wave learns its sorted count here (a query flagged by the filter
// keeps none: the host runs it again).
__global__ __launch_bounds__(kBlock) void k_hit_compact(const uint64_t *__restrict__ keys,
                                                        const uint32_t *__restrict__ hrel,
                                                        const int64_t *__restrict__ qoff,
                                                        int32_t qa, int64_t g0, int32_t nqw,
                                                        const uint32_t *__restrict__ kept,
                                                        const uint32_t *__restrict__ koff,
                                                        uint64_t *__restrict__ out,
                                                        WaveCtl *__restrict__ ctl)
{
    // koff null: each block adds up the kept counts before its own (few queries)
    if (ctl) {
        qa = ctl->qa;
        g0 = ctl->g0;
        nqw = ctl->nqw;
        if (blockIdx.x == 0) {
            const uint32_t total = koff ? koff[nqw] : block_sum(kept, (uint32_t)nqw);
            if (threadIdx.x == 0) ctl->H = total;
        }
    }
    const int32_t ql = (int32_t)blockIdx.x;
    if (ql >= nqw) return;
    const uint64_t *src = keys + hrel[qoff[qa + ql] - g0];
    uint64_t *dst = out + (koff ? koff[ql] : block_sum(kept, (uint32_t)ql));
    const uint32_t n = kept[ql];
    for (uint32_t i = threadIdx.x; i < n; i += kBlock) dst[i] = src[i];
}

void launch_hit_filter(uint64_t *keys, const uint32_t *hrel, const int64_t *qoff, int32_t qa,
                       int64_t g0, int32_t nqw, int bp, const int32_t *order, uint32_t *kept,
                       uint32_t *flag, hipStream_t st, WaveCtl *ctl, int32_t nq_cap)
{
    const int32_t nb = ctl ? nq_cap : nqw;
    if (nb > 0)
        k_hit_filter<<<nb, kFiltBlock, 0, st>>>(keys, hrel, qoff, qa, g0, nqw, bp, order, kept,
                                                flag, ctl);
}

void launch_gather_filter(const uint32_t *hrel, const uint32_t *pbase, const int2 *post, const int64_t *qoff, int32_t qa, int64_t g0,
                          int32_t nqw, HitKeyLayout lay, const int32_t *order, uint64_t *keys,
                          uint32_t *kept, uint32_t *flag, hipStream_t st, WaveCtl *ctl,
                          int32_t nq_cap)
{
    const int32_t nb = ctl ? nq_cap : nqw;
    if (nb > 0)
        k_gather_filter<<<nb, kFiltBlock, 0, st>>>(hrel, pbase, post, qoff, qa, g0, nqw, lay,
                                                   order, keys, kept, flag, ctl);
}

void launch_hit_compact(const uint64_t *keys, const uint32_t *hrel, const int64_t *qoff,
                        int32_t qa, int64_t g0, int32_t nqw, const uint32_t *kept, uint32_t *koff,
                        uint32_t *partials, uint64_t *out, hipStream_t st, WaveCtl *ctl,
                        int32_t nq_cap)
{
    const int32_t nb = ctl ? nq_cap : nqw;
    if (nb <= 0) return;
    // a replayed wave of a few thousand queries skips the scan: blocks add up
    // the counts before them
    const bool self = ctl && nq_cap <= 4096;
    if (!self) launch_scan_u32(kept, koff, nb, partials, st);
    k_hit_compact<<<nb, kBlock, 0, st>>>(keys, hrel, qoff, qa, g0, nqw, kept, self ? nullptr : koff,
                                         out, ctl);
}

// ------------------------------------------------------------------ S5: chain + filter
// A sorted hit ends a run when the next hit is in another (q, s, diag) group or
// more than G past this hit's window; the run's first hit is found by walking back
// while the chaining rule holds (in the tile's LDS copy, then in global memory).
// Runs with qe - qs >= M are kept.  Two passes over tiles of hits (count, then
// write after a scan of the tile counts) keep the runs in hit-key order, so they
// come out grouped by query and sequence.
//
// The tile's keys are staged in LDS: s_k[1 + l] is key base + l for l < cnt, and
// s_k[cnt + 1] the key after the tile (when base + cnt < n).  Hit a chains to the
// next hit b when both lie in one (q, s, diag) group and b's window starts at most
// G past a's window.
__device__ __forceinline__ bool chains_to(uint64_t a, uint64_t b, int bp, int32_t k, int32_t G)
{
    const uint64_t pmask = low_mask(bp);
    return (a >> bp) == (b >> bp) && (int32_t)(b & pmask) - ((int32_t)(a & pmask) + k) <= G;
}

// qs[r] = qpos of the first hit of the run that tile hit l = r kBlock + t (thread
// t's r-th item) belongs to, in the thread's registers.  Starts
// inside the tile come from a running maximum of start positions over the tile's
// 32 chunks of 64 hits (chunk 4 r + w is wave w's r-th row of the block's items,
// so each wave scans its own rows and the chunks' maxima are combined once); the
// run that enters the tile from before it is walked back once, by wave 0, 64 keys
// at a time.
__device__ void tile_run_starts(const uint64_t *__restrict__ s_k,
                                const uint64_t *__restrict__ keys, uint32_t base, uint32_t cnt,
                                int bp, int32_t k, int32_t G, int32_t (&qs)[kItems])
{
    constexpr int kChunks = kItems * (kBlock / 64);
    __shared__ int32_t s_carry;
    __shared__ int32_t s_cm[kChunks];
    const uint64_t pmask = low_mask(bp);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const bool enters = cnt > 0 && base > 0 && chains_to(keys[base - 1], s_k[1], bp, k, G);
    if (threadIdx.x < 64 && enters) {
        for (uint32_t c = 0;; c += 64) {
            // key j = base - 1 - c - lane starts the run unless key j - 1 chains to it
            const int64_t j = (int64_t)base - 1 - c - lane;
            bool first = false;
            if (j >= 0) first = j == 0 || !chains_to(keys[j - 1], keys[j], bp, k, G);
            const uint64_t m = __ballot(first);
            if (m) {
                const int f = __ffsll((unsigned long long)m) - 1;
                if (lane == f) s_carry = (int32_t)(keys[j] & pmask);
                break;
            }
        }
    }
    int32_t st[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const uint32_t l = r * kBlock + threadIdx.x;
        bool start = false;
        if (l < cnt) start = l == 0 ? !enters : !chains_to(s_k[l], s_k[1 + l], bp, k, G);
        int32_t x = start ? (int32_t)l : -1;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x = max(x, y);
        }
        st[r] = x;
        if (lane == 63) s_cm[r * (kBlock / 64) + w] = x;
    }
    __syncthreads();  // s_cm and s_carry are set
    // exclusive maximum of the chunk maxima, chunk c in lane c
    int32_t cm = lane < kChunks ? s_cm[lane] : -1;
#pragma unroll
    for (int o = 1; o < kChunks; o <<= 1) {
        const int32_t y = __shfl_up(cm, o, 64);
        if (lane >= o) cm = max(cm, y);
    }
    int32_t ex = __shfl_up(cm, 1, 64);
    if (lane == 0) ex = -1;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const uint32_t l = r * kBlock + threadIdx.x;
        const int32_t before = __shfl(ex, r * (kBlock / 64) + w, 64);
        qs[r] = 0;
        if (l < cnt) {
            const int32_t a = max(st[r], before);
            qs[r] = a >= 0 ? (int32_t)(s_k[1 + a] & pmask) : s_carry;
        }
    }
    __syncthreads();
}

// Tile hit l ends a run when the next hit does not chain to it; the run [qs, qe =
// qpos + k) is kept when qe - qs >= M.
__device__ __forceinline__ bool chain_end_tile(const uint64_t *__restrict__ s_k, int32_t qs,
                                               uint32_t n, uint32_t base, uint32_t l, int bp,
                                               int32_t k, int32_t G, int32_t M)
{
    const uint64_t key = s_k[1 + l];
    if (base + l + 1 < n && chains_to(key, s_k[2 + l], bp, k, G)) return false;
    return (int32_t)(key & low_mask(bp)) + k - qs >= M;
}

// Stage keys [base, base + cnt] (the tile and the key after it) in LDS.
__device__ __forceinline__ uint32_t stage_chain_tile(const uint64_t *__restrict__ keys, uint32_t n,
                                                     uint32_t base, uint64_t *__restrict__ s_k)
{
    const uint32_t cnt = base < n ? min((uint32_t)kTile, n - base) : 0u;
    // two keys per 16-byte load (tile starts are multiples of kTile keys)
#pragma unroll
    for (int r = 0; r < kItems / 2; ++r) {
        const uint32_t l = 2 * (r * kBlock + threadIdx.x);
        if (l + 1 < cnt) {
            const u64x2_a8 v = *reinterpret_cast<const u64x2_a8 *>(keys + base + l);
            s_k[1 + l] = v.x;
            s_k[2 + l] = v.y;
        } else if (l < cnt) {
            s_k[1 + l] = keys[base + l];
        }
    }
    if (threadIdx.x == 0 && base + cnt < n) s_k[cnt + 1] = keys[base + cnt];
    __syncthreads();
    return cnt;
}

__global__ __launch_bounds__(kBlock) void k_chain_count(const uint64_t *__restrict__ keys,
                                                        uint32_t n, int bp, int32_t k, int32_t G,
                                                        int32_t M, uint32_t *__restrict__ counts,
                                                        const WaveCtl *__restrict__ ctl)
{
    __shared__ uint64_t s_k[kTile + 2];
    if (ctl) {  // tiles past the wave's hits count zero runs
        n = ctl->H;
        bp = ctl->lay.bp;
    }
    const uint32_t base = blockIdx.x * (uint32_t)kTile;
    const uint32_t cnt = stage_chain_tile(keys, n, base, s_k);
    int32_t qs[kItems];
    tile_run_starts(s_k, keys, base, cnt, bp, k, G, qs);
    uint32_t c = 0;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const uint32_t l = r * kBlock + threadIdx.x;
        if (l < cnt && chain_end_tile(s_k, qs[r], n, base, l, bp, k, G, M)) ++c;
    }
    uint32_t tot;
    block_excl_scan<uint32_t>(c, &tot);
    if (threadIdx.x == 0) counts[blockIdx.x] = tot;
}

// SELF (replayed waves with few hits): no scan of the tile counts; each tile with
// hits adds up the counts before it, and the last one stores the total in ctl->nc.
template <bool SELF>
__global__ __launch_bounds__(kBlock) void k_chain_write(const uint64_t *__restrict__ keys,
                                                        uint32_t n, HitKeyLayout lay, int32_t k,
                                                        int32_t G, int32_t M,
                                                        const uint32_t *__restrict__ tile_off,
                                                        Cand *__restrict__ out,
                                                        WaveCtl *__restrict__ ctl)
{
    if (ctl) {
        n = ctl->H;
        lay = ctl->lay;
    }
    const uint32_t base = blockIdx.x * (uint32_t)kTile;
    if (SELF && n == 0 && blockIdx.x == 0 && threadIdx.x == 0) ctl->nc = 0;
    if (ctl && base >= n) return;
    __shared__ uint64_t s_k[kTile + 2];
    const uint32_t cnt = stage_chain_tile(keys, n, base, s_k);
    int32_t qsv[kItems];
    tile_run_starts(s_k, keys, base, cnt, lay.bp, k, G, qsv);
    uint32_t at = SELF ? block_sum(tile_off, blockIdx.x) : tile_off[blockIdx.x];
    // runs in hit order: row r of wave w is chunk 4 r + w; one scan of the chunks'
    // run counts places every run
    constexpr int kChunks = kItems * (kBlock / 64);
    __shared__ uint32_t s_cc[kChunks];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t below = (1ull << lane) - 1ull;
    uint64_t em[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const uint32_t l = r * kBlock + threadIdx.x;
        const bool emit = l < cnt && chain_end_tile(s_k, qsv[r], n, base, l, lay.bp, k, G, M);
        em[r] = __ballot(emit);
        if (lane == 0) s_cc[r * (kBlock / 64) + w] = (uint32_t)__popcll(em[r]);
    }
    __syncthreads();
    uint32_t cc = lane < kChunks ? s_cc[lane] : 0u;
#pragma unroll
    for (int o = 1; o < kChunks; o <<= 1) {
        const uint32_t y = __shfl_up(cc, o, 64);
        if (lane >= o) cc += y;
    }
    const uint32_t total = __shfl(cc, kChunks - 1, 64);
    uint32_t ex = __shfl_up(cc, 1, 64);
    if (lane == 0) ex = 0;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const uint32_t l = r * kBlock + threadIdx.x;
        const uint32_t chunk_at = __shfl(ex, r * (kBlock / 64) + w, 64);
        if ((em[r] >> lane) & 1ull) {
            const uint64_t key = s_k[1 + l];
            const uint64_t grp = key >> lay.bp;
            Cand c;
            c.d = (int32_t)(grp & low_mask(lay.bd)) - lay.bias;
            c.s = (int32_t)(shr64(grp, lay.bd) & low_mask(lay.bs));
            c.q = (int32_t)shr64(grp, lay.bd + lay.bs);
            c.qs = qsv[r];
            c.qe = (int32_t)(key & low_mask(lay.bp)) + k;
            out[at + chunk_at + (uint32_t)__popcll(em[r] & below)] = c;
        }
    }
    at += total;
    if (SELF && base + kTile >= n && threadIdx.x == 0) ctl->nc = at;  // the last tile
}

void launch_chain_count(const uint64_t *keys, uint32_t n, HitKeyLayout lay, int32_t k,
                        int32_t max_gap, int32_t min_len, uint32_t *counts, hipStream_t st)
{
    if (n == 0) return;
    k_chain_count<<<(n + kTile - 1) / kTile, kBlock, 0, st>>>(keys, n, lay.bp, k, max_gap, min_len,
                                                              counts, nullptr);
}

void launch_chain_write(const uint64_t *keys, uint32_t n, HitKeyLayout lay, int32_t k,
                        int32_t max_gap, int32_t min_len, const uint32_t *tile_off, Cand *out,
                        hipStream_t st)
{
    if (n == 0) return;
    k_chain_write<false><<<(n + kTile - 1) / kTile, kBlock, 0, st>>>(keys, n, lay, k, max_gap, min_len,
                                                              tile_off, out, nullptr);
}

// Chaining of a graph-replayed wave over tiles of hits_cap hits: run counts per
// tile, their scan (total at counts[tiles], copied to ctl->nc), then the runs.
// With few hits (the lone-diagonal filter ran) the write kernel adds up the
// counts of the tiles before it instead.
void launch_chain_ctl(const uint64_t *keys, uint32_t hits_cap, int32_t k, int32_t max_gap,
                      int32_t min_len, uint32_t *counts, uint32_t *partials, Cand *out,
                      WaveCtl *ctl, hipStream_t st, bool few)
{
    const uint32_t nt = std::max<uint32_t>(1, (hits_cap + kTile - 1) / kTile);
    k_chain_count<<<nt, kBlock, 0, st>>>(keys, 0, 0, k, max_gap, min_len, counts, ctl);
    if (few) {
        k_chain_write<true><<<nt, kBlock, 0, st>>>(keys, 0, HitKeyLayout{}, k, max_gap, min_len,
                                                   counts, out, ctl);
        return;
    }
    scan_impl<uint32_t, uint32_t>(counts, counts, nt, partials, st, &ctl->nc);
    k_chain_write<false><<<nt, kBlock, 0, st>>>(keys, 0, HitKeyLayout{}, k, max_gap, min_len,
                                                counts, out, ctl);
}

// Runs come out in (q, s, diag) order: each query's runs are one range
// [qstart, qend), found at its boundaries (no per-run counter, no atomics).
// Query q's runs are [qstart[q], qend[q]): the first run of a query >= q and of a
// query >= q + 1, by binary search over the runs' query fields (one thread per
// query; a query without runs gets an empty range).
__global__ void k_cand_segments(const Cand *__restrict__ c, uint32_t n, int32_t nq,
                                uint32_t *__restrict__ qstart, uint32_t *__restrict__ qend)
{
    const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    auto first_at_least = [&](int32_t v) {
        uint32_t a = 0, b = n;
        while (a < b) {
            const uint32_t mid = a + ((b - a) >> 1);
            if (c[mid].q < v) a = mid + 1;
            else b = mid;
        }
        return a;
    };
    qstart[q] = first_at_least(q);
    qend[q] = first_at_least(q + 1);
}

void launch_cand_segments(const Cand *c, uint32_t n, int32_t nq, uint32_t *qstart, uint32_t *qend,
                          hipStream_t st)
{
    if (nq > 0)
        k_cand_segments<<<(uint32_t)((nq + kBlock - 1) / kBlock), kBlock, 0, st>>>(c, n, nq, qstart,
                                                                                qend);
}

uint32_t chain_tiles(uint32_t n) { return (n + kTile - 1) / kTile; }

// ------------------------------------------------------------------ S6: X-drop extension
// One wave per run and side.  The walk is taken 64 steps at a time: each lane
// scores one step, a wave prefix sum gives the running sums, a prefix maximum the
// best-so-far, and the first lane whose sum is more than X below that best ends
// the walk.  The extension is the first step at the best sum (strictly above the
// best of earlier steps), exactly as a step-by-step walk finds it.
__device__ __forceinline__ int32_t wave_incl_sum(int32_t x, int lane)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

__device__ __forceinline__ int32_t wave_incl_max(int32_t x, int lane)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x = max(x, y);
    }
    return x;
}

__device__ __forceinline__ int32_t wave_max(int32_t x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o, 64));
    return x;
}

// Steps s = 0 .. T-1 score query base from + s (right) or from - 1 - s (left)
// against data-bank base at the same query position + d.  The walk may resume at
// step t0 with its running sum, best sum and best step so far.
template <bool RIGHT>
__device__ __forceinline__ int32_t xdrop_side(const uint8_t *__restrict__ q,
                                              const uint32_t *__restrict__ dbw, int64_t s0,
                                              int32_t from, int32_t d, int32_t T, int32_t match,
                                              int32_t mismatch, int32_t X, int lane,
                                              int32_t t0 = 0, int32_t run = 0, int32_t best = 0,
                                              int32_t bl = 0)
{
    for (int32_t base = t0; base < T; base += 64) {
        const int32_t step = base + lane;
        const bool valid = step < T;
        int32_t v = 0;
        if (valid) {
            const int32_t qi = RIGHT ? from + step : from - 1 - step;
            v = ((int32_t)q[qi] == db_base(dbw, s0 + qi + d)) ? match : -mismatch;
        }
        const int32_t r = run + wave_incl_sum(v, lane);
        const int32_t bt = max(best, wave_incl_max(r, lane));
        const uint64_t sm = __ballot(valid && (bt - r > X));
        const int32_t lim = sm ? (__ffsll((unsigned long long)sm) - 1) : min(63, T - 1 - base);
        const bool in = lane <= lim;
        const int32_t m = wave_max(in ? r : INT32_MIN);
        if (m > best) {
            const uint64_t am = __ballot(in && r == m);
            best = m;
            bl = base + __ffsll((unsigned long long)am);  // first step (1-based) at the best
        }
        run = __shfl(r, lim, 64);
        if (sm) break;
    }
    return bl;
}

// The same walk one step at a time in one lane, for at most `cap` steps (bases
// read four steps ahead; the data-bank word is kept while the walk stays in it).
// Returns true when the walk ended (drop over X, or the sequence or query end);
// otherwise (t, run, best, bl) hold the state after `cap` steps.
template <bool RIGHT>
__device__ __forceinline__ bool xdrop_lane(const uint8_t *__restrict__ q,
                                           const uint32_t *__restrict__ dbw, int64_t s0,
                                           int32_t from, int32_t d, int32_t T, int32_t match,
                                           int32_t mismatch, int32_t X, int32_t cap, int32_t &t,
                                           int32_t &run, int32_t &best, int32_t &bl)
{
    t = 0;
    run = 0;
    best = 0;
    bl = 0;
    const int32_t end = min(T, cap);
    int64_t wi = -1;
    uint32_t word = 0;
    while (t < end) {
        int32_t qb[4], db[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            qb[u] = -1;
            db[u] = -2;
            if (t + u < end) {
                const int32_t qi = RIGHT ? from + t + u : from - 1 - (t + u);
                const int64_t g = s0 + qi + d;
                if ((g >> 4) != wi) {
                    wi = g >> 4;
                    word = dbw[wi];
                }
                qb[u] = q[qi];
                db[u] = (int32_t)((word >> (30u - ((uint32_t)(g & 15) << 1))) & 3u);
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (t >= end) break;
            run += qb[u] == db[u] ? match : -mismatch;
            ++t;
            if (run > best) {
                best = run;
                bl = t;
            }
            if (best - run > X) return true;
        }
    }
    return t >= T;
}

// Extension in two kernels.  k_extend walks both sides of every run in one lane
// for up to lane_steps steps (0: none), which ends most walks in random sequence;
// the state of a walk still going is queued, and k_extend_long resumes each
// queued walk with a whole wave, 64 steps at a time.  A full queue makes the lane
// finish its own walk.
struct XWalk {
    uint32_t run_ix;  // index of the run; bit 31 set for the left side
    int32_t t, run, best, bl;
};

// Queue slot of this lane's walk if `need` (one atomic per wave: the lanes that
// need a slot take consecutive ones).
__device__ __forceinline__ uint32_t queue_slot(bool need, uint32_t *__restrict__ qcount, int lane)
{
    const uint64_t m = __ballot(need);
    if (m == 0) return 0;
    const int leader = __ffsll((unsigned long long)m) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(qcount, (uint32_t)__popcll(m));
    base = __shfl(base, leader, 64);
    return base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
}

// The batch's query codes packed 16 to a word like the data bank (first base in
// the top bits), for the extension's word compares; two spare words at the end.
__global__ void k_pack_query(const uint8_t *__restrict__ qcode, int64_t T,
                             uint32_t *__restrict__ qpack, int64_t nwords)
{
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nwords) return;
    uint32_t v = 0;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int64_t g = 16 * w + t;
        const uint32_t c = g < T ? (uint32_t)(qcode[g] & 3u) : 0u;
        v |= c << (30 - 2 * t);
    }
    qpack[w] = v;
}

void launch_pack_query(const uint8_t *qcode, int64_t T, uint32_t *qpack, hipStream_t st)
{
    const int64_t nwords = (T + 15) / 16 + 2;
    k_pack_query<<<(uint32_t)((nwords + kBlock - 1) / kBlock), kBlock, 0, st>>>(qcode, T, qpack,
                                                                             nwords);
}

// 16 bases of a 2-bit packed array (first base in the top bits) starting at g,
// first base in bits 31:30.  Reads words g / 16 and g / 16 + 1.
__device__ __forceinline__ uint32_t bases16_from(const uint32_t *__restrict__ w, int64_t g)
{
    const int64_t wi = g >> 4;
    const uint64_t v = ((uint64_t)w[wi] << 32) | (uint64_t)w[wi + 1];
    return (uint32_t)(v >> (32u - ((uint32_t)(g & 15) << 1)));
}

// The 16 bases before position p (p - 16 .. p - 1), base p - 1 in bits 1:0.  Below
// p = 16 the missing bases read as zero; a walk never consumes them.
__device__ __forceinline__ uint32_t bases16_before(const uint32_t *__restrict__ w, int64_t p)
{
    if (p >= 16) return bases16_from(w, p - 16);
    return p <= 0 ? 0u : (bases16_from(w, 0) >> (2u * (uint32_t)(16 - p)));
}

// X-drop walk of one lane, 16 steps per chunk.  The query and data-bank bases of
// the chunk's 16 steps are read as packed words, compared at once (a 2-bit XOR),
// and the running sum moves from one mismatch to the next: between mismatches it
// only rises, so its maximum over a stretch of matches is at the stretch's end
// (the first step at that value), and it can only fall more than X below the best
// at a mismatch.  This is the step-by-step rule exactly.  xdrop_x reads a chunk's
// XOR word (t < T: the walk's own bases).
template <bool RIGHT>
__device__ __forceinline__ uint32_t xdrop_x(const uint32_t *__restrict__ qpack, int64_t gq,
                                            const uint32_t *__restrict__ dbw, int64_t gb,
                                            int32_t t)
{
    // RIGHT: step i (0-based) is the base in bits 31-2i:30-2i; otherwise in bits 2i+1:2i
    return RIGHT ? bases16_from(qpack, gq + t) ^ bases16_from(dbw, gb + t)
                 : bases16_before(qpack, gq - t) ^ bases16_before(dbw, gb - t);
}

// The chunk's XOR word for a walk of either side, step i in bits 2i+1:2i.  A left
// walk's word is read 16 positions lower, its first step (the base nearest the
// run) in the low bits; a right walk's word is bit-reversed into the same order.
// Both sides of a wave's walks then take one code path.
__device__ __forceinline__ uint32_t xdrop_xw(const uint32_t *__restrict__ qpack, int64_t gq,
                                             const uint32_t *__restrict__ dbw, int64_t gb,
                                             int32_t t, bool left)
{
    const int64_t pq = left ? gq - t - 16 : gq + t, pb = left ? gb - t - 16 : gb + t;
    uint32_t x;
    if (pq >= 0 && pb >= 0) x = bases16_from(qpack, pq) ^ bases16_from(dbw, pb);
    else x = xdrop_x<false>(qpack, gq, dbw, gb, t);  // a left walk near the arrays' starts
    return left ? x : __brev(x);
}

// One chunk of a walk (t < T): the up to 16 steps from t, whose query and bank
// bases differ where the 2-bit XOR x is non-zero (step i in bits 2i+1:2i).  Each
// turn of the loop takes the stretch of matches up to the next mismatch (the
// running sum's maximum over it is at its end) and then that mismatch, whose drop
// is tested; past the chunk's last mismatch the stretch runs to the chunk's end.
// Returns true when the walk ended (drop over X, or T steps); otherwise t has
// moved 16 steps on.  SMALL: match < 2^24, so a stretch's gain (at most 16
// matches) takes a 24-bit multiply.
template <bool SMALL>
__device__ __forceinline__ bool xdrop_chunk(uint32_t x, int32_t T, int32_t match,
                                            int32_t mismatch, int32_t X, int32_t &t, int32_t &run,
                                            int32_t &best, int32_t &bl)
{
    const int32_t nstep = min(16, T - t);
    uint32_t mm = (x | (x >> 1)) & 0x55555555u;  // one flag bit per step
    if (nstep < 16) mm &= (1u << (2 * nstep)) - 1u;
    int32_t pos = 0, nx, blx = -1;  // blx: the chunk's step at a new best, if any
    bool drop;
    do {
        nx = mm ? (int32_t)(__builtin_ctz(mm) >> 1) : nstep;  // the next mismatch
        run += SMALL ? (int32_t)__umul24((uint32_t)(nx - pos), (uint32_t)match) : (nx - pos) * match;
        blx = run > best ? nx : blx;  // first step at a new best
        best = max(best, run);
        run -= mismatch;  // undone below when the chunk had no mismatch left
        drop = best - run > X;
        mm &= mm - 1u;
        pos = nx + 1;
    } while (nx < nstep && !drop);
    if (blx >= 0) bl = t + blx;
    if (nx >= nstep) {
        run += mismatch;
        t += nstep;
        return t >= T;
    }
    t += nx + 1;
    return true;
}

// Extension of every run on both sides (Section 2.2 phase 3).  Each side of each
// run is one walk; whole waves take contiguous ranges of walks, and a lane whose
// walk ends takes the next one of its wave's range at once, so lanes do not idle
// behind the longest walk of a group.  A walk still going after `lane_steps`
// steps is queued (its state saved) and k_extend_long resumes it with a whole
// wave; a full queue makes the lane finish the walk itself.  The right walk of a
// run writes its box's run fields and right end, the left walk its left end; a
// queued side is rewritten by k_extend_long.
__global__ __launch_bounds__(kBlock) void k_extend(const Cand *__restrict__ cands, uint32_t n,
                                                   const uint32_t *__restrict__ qpack,
                                                   const int64_t *__restrict__ qoff, int32_t qa,
                                                   const uint32_t *__restrict__ dbw,
                                                   const int64_t *__restrict__ seq_start,
                                                   int32_t match, int32_t mismatch, int32_t X,
                                                   Box *__restrict__ out, XWalk *__restrict__ queue,
                                                   uint32_t qcap, uint32_t *__restrict__ qcount,
                                                   int32_t lane_steps, const WaveCtl *__restrict__ ctl)
{
    if (ctl) {
        n = ctl->nc;
        qa = ctl->qa;
    }
    const int lane = threadIdx.x & 63;
    const uint64_t nwave = (uint64_t)gridDim.x * (kBlock / 64);
    const uint64_t wave = (uint64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const uint64_t items = 2ull * n;  // walk w: run w / 2, left side when w is odd
    const uint64_t per = (items + nwave - 1) / nwave;
    uint64_t next = wave * per;
    const uint64_t stop = min(items, next + per);
    const uint64_t below = (1ull << lane) - 1ull;
    bool have = false, left = false;
    uint32_t ri = 0;
    Cand c{0, 0, 0, 0, 0};
    int64_t gq = 0, gb = 0;
    int32_t T = 0, t = 0, run = 0, best = 0, bl = 0, cap = 0;
    uint32_t xn = 0;   // the bases' XOR of a going walk's next chunk, when xok
    bool xok = false;
    for (;;) {
        // lanes without a walk take the next walks of the wave's range
        const uint64_t need = __ballot(!have);
        if (need && next < stop) {
            if (!have) {
                const uint64_t w = next + (uint64_t)__popcll(need & below);
                if (w < stop) {
                    have = true;
                    ri = (uint32_t)(w >> 1);
                    left = (w & 1) != 0;
                    c = cands[ri];
                    const int64_t q0 = qoff[qa + c.q];
                    const int32_t L = (int32_t)(qoff[qa + c.q + 1] - q0);
                    const int64_t s0 = seq_start[c.s];
                    const int32_t ns = (int32_t)(seq_start[c.s + 1] - s0);
                    if (left) {
                        T = min(c.qs, c.qs + c.d);
                        gq = q0 + c.qs;
                        gb = s0 + c.qs + c.d;
                    } else {
                        T = min(L - c.qe, ns - (c.qe + c.d));
                        gq = q0 + c.qe;
                        gb = s0 + c.qe + c.d;
                    }
                    t = run = best = bl = 0;
                    cap = lane_steps;
                }
            }
            next += (uint64_t)__popcll(need);
        }
        if (__ballot(have) == 0) break;
        // one 16-step chunk of every walk per round, so that a lane whose walk ends
        // takes its next walk without waiting for the longest walk of the wave; a
        // walk that goes on has its next chunk's bases read at the end of the round,
        // so the reads overlap the other lanes' refills
        bool done = false, park = false;
        if (have) {
            if (t >= T) {
                done = true;
            } else if (t >= cap) {
                park = true;  // past the lane's cap: to the queue for a whole wave
            } else {
                const uint32_t x = xok ? xn : xdrop_xw(qpack, gq, dbw, gb, t, left);
                done = match < (1 << 24)
                           ? xdrop_chunk<true>(x, T, match, mismatch, X, t, run, best, bl)
                           : xdrop_chunk<false>(x, T, match, mismatch, X, t, run, best, bl);
            }
        }
        xok = false;
        const uint32_t slot = queue_slot(park, qcount, lane);
        const bool queued = park && slot < qcap;
        if (queued) queue[slot] = XWalk{ri | (left ? 0x80000000u : 0u), t, run, best, bl};
        if (park && !queued) cap = INT32_MAX;  // queue full: this lane finishes the walk
        if (have && !done && !queued && t < cap) {
            xn = xdrop_xw(qpack, gq, dbw, gb, t, left);
            xok = true;
        }
        if (done || queued) {
            Box *b = out + ri;
            if (left) {
                b->qs = c.qs - bl;
                b->ds = c.qs - bl + c.d;
            } else {
                b->q = c.q;
                b->s = c.s;
                b->qe = c.qe + bl;
                b->de = c.qe + bl + c.d;
                b->dmin = c.d;
                b->dmax = c.d;
            }
            have = false;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_extend_long(const Cand *__restrict__ cands,
                                                        const uint8_t *__restrict__ qcode,
                                                        const int64_t *__restrict__ qoff,
                                                        int32_t qa,
                                                        const uint32_t *__restrict__ dbw,
                                                        const int64_t *__restrict__ seq_start,
                                                        int32_t match, int32_t mismatch, int32_t X,
                                                        Box *__restrict__ out,
                                                        const XWalk *__restrict__ queue,
                                                        uint32_t qcap,
                                                        const uint32_t *__restrict__ qcount,
                                                        const WaveCtl *__restrict__ ctl)
{
    if (ctl) qa = ctl->qa;
    const int lane = threadIdx.x & 63;
    const uint32_t nw = min(*qcount, qcap);
    for (uint32_t e = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); e < nw;
         e += gridDim.x * (kBlock / 64)) {  // whole waves
        const XWalk w = queue[e];
        const bool left = (w.run_ix >> 31) != 0;
        const uint32_t i = w.run_ix & 0x7fffffffu;
        const Cand c = cands[i];
        const int64_t q0 = qoff[qa + c.q];
        const int32_t L = (int32_t)(qoff[qa + c.q + 1] - q0);
        const uint8_t *__restrict__ q = qcode + q0;
        const int64_t s0 = seq_start[c.s];
        const int32_t ns = (int32_t)(seq_start[c.s + 1] - s0);
        const int32_t d = c.d;
        if (left) {
            const int32_t tl = min(c.qs, c.qs + d);
            const int32_t el = xdrop_side<false>(q, dbw, s0, c.qs, d, tl, match, mismatch, X, lane,
                                                 w.t, w.run, w.best, w.bl);
            if (lane == 0) {
                out[i].qs = c.qs - el;
                out[i].ds = c.qs - el + d;
            }
        } else {
            const int32_t tr = min(L - c.qe, ns - (c.qe + d));
            const int32_t er = xdrop_side<true>(q, dbw, s0, c.qe, d, tr, match, mismatch, X, lane,
                                                w.t, w.run, w.best, w.bl);
            if (lane == 0) {
                out[i].qe = c.qe + er;
                out[i].de = c.qe + er + d;
            }
        }
    }
}

size_t extend_queue_bytes(uint32_t n)
{
    return sizeof(XWalk) * (size_t)std::min<uint32_t>(std::max<uint32_t>(n, 1u), 1u << 22) +
           256;
}

void launch_extend(const Cand *c, uint32_t n, const uint8_t *qcode, const uint32_t *qpack,
                   const int64_t *qoff, int32_t qa, const uint32_t *dbw, const int64_t *seq_start,
                   int32_t match, int32_t mismatch, int32_t xdrop, Box *out, void *queue_mem,
                   int32_t lane_steps, hipStream_t st, const WaveCtl *ctl, uint32_t n_cap,
                   bool count_cleared)
{
    // graph form: n comes from ctl, grids are sized for n_cap runs
    const uint32_t nmax = ctl ? n_cap : n;
    if (nmax == 0) return;
    uint32_t *qcount = static_cast<uint32_t *>(queue_mem);
    XWalk *queue = reinterpret_cast<XWalk *>(static_cast<char *>(queue_mem) + 256);
    const uint32_t qcap = (uint32_t)((extend_queue_bytes(nmax) - 256) / sizeof(XWalk));
    if (!count_cleared) launch_fill_u32(qcount, 1, 0u, st);
    // one wave per 64 walks up to 8 waves per SIMD on every CU; beyond that each
    // wave's range grows
    const uint32_t nb = ctl ? kStrideGrid
                            : (uint32_t)std::min<uint64_t>((2ull * n + kBlock - 1) / kBlock, 8192);
    k_extend<<<nb, kBlock, 0, st>>>(c, n, qpack, qoff, qa, dbw, seq_start, match, mismatch, xdrop,
                                    out, queue, qcap, qcount, std::max(lane_steps, 0), ctl);
    const uint64_t most = std::min<uint64_t>(2ull * nmax, qcap);  // queued walks at most
    const uint32_t lb = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((most + 3) / 4, 1u << 16));
    k_extend_long<<<lb, kBlock, 0, st>>>(c, qcode, qoff, qa, dbw, seq_start, match, mismatch,
                                         xdrop, out, queue, qcap, qcount, ctl);
}

// ------------------------------------------------------------------ record sort keys
__device__ __forceinline__ uint64_t box_field(const Box &b, int32_t f, int32_t desc_max)
{
    switch (f) {
    case F_Q: return (uint32_t)b.q;
    case F_S: return (uint32_t)b.s;
    case F_QS: return (uint32_t)b.qs;
    case F_QE: return (uint32_t)b.qe;
    case F_DS: return (uint32_t)b.ds;
    case F_DE: return (uint32_t)b.de;
    default: return (uint32_t)(desc_max - min(b.qe - b.qs, b.de - b.ds));
    }
}

__global__ void k_box_keys(const Box *__restrict__ b, uint32_t n, KeyWord w, int32_t q_invalid,
                           uint64_t *__restrict__ out, const uint32_t *__restrict__ perm)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Box x = b[perm ? perm[i] : i];
    if (x.q < 0) x = Box{q_invalid, 0, 0, 0, 0, 0, 0, 0};
    uint64_t key = 0;
    for (int f = 0; f < w.n; ++f) key |= box_field(x, w.field[f], w.desc_max[f]) << w.shift[f];
    out[i] = key;
}

void launch_box_keys(const Box *b, uint32_t n, KeyWord w, int32_t q_invalid, uint64_t *out,
                     const uint32_t *perm, hipStream_t st)
{
    if (n == 0) return;
    k_box_keys<<<(n + kBlock - 1) / kBlock, kBlock, 0, st>>>(b, n, w, q_invalid, out, perm);
}

__device__ __forceinline__ uint64_t align_field(const Align &a, int32_t f, int32_t desc_max)
{
    switch (f) {
    case A_Q: return (uint32_t)a.q;
    case A_SCORE_DESC: return (uint32_t)(desc_max - a.score);
    case A_SEQ: return (uint32_t)a.seq_id;
    case A_QS: return (uint32_t)a.q_start;
    case A_QE: return (uint32_t)a.q_end;
    case A_DS: return (uint32_t)a.d_start;
    case A_DE: return (uint32_t)a.d_end;
    case A_BQS: return (uint32_t)a.box_q_start;
    case A_BQE: return (uint32_t)a.box_q_end;
    case A_BDS: return (uint32_t)a.box_d_start;
    case A_D0: return (uint32_t)(a.band_d0 + desc_max);
    default: return (uint32_t)a.box_d_end;
    }
}

__global__ void k_align_keys(const Align *__restrict__ a, uint32_t n, KeyWord w, int32_t q_invalid,
                             uint64_t *__restrict__ out, const uint32_t *__restrict__ perm)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Align x = a[perm ? perm[i] : i];
    uint64_t key = 0;
    if (x.score <= 0) {
        for (int f = 0; f < w.n; ++f)
            if (w.field[f] == A_Q) key |= (uint64_t)(uint32_t)q_invalid << w.shift[f];
    } else {
        for (int f = 0; f < w.n; ++f) key |= align_field(x, w.field[f], w.desc_max[f]) << w.shift[f];
    }
    out[i] = key;
}

void launch_align_keys(const Align *a, uint32_t n, KeyWord w, int32_t q_invalid, uint64_t *out,
                       const uint32_t *perm, hipStream_t st)
{
    if (n == 0) return;
    k_align_keys<<<(n + kBlock - 1) / kBlock, kBlock, 0, st>>>(a, n, w, q_invalid, out, perm);
}

__global__ void k_iota(uint32_t *__restrict__ v, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = i;
}

void launch_iota(uint32_t *v, uint32_t n, hipStream_t st)
{
    if (n) k_iota<<<(n + kBlock - 1) / kBlock, kBlock, 0, st>>>(v, n);
}

template <typename R>
__global__ void k_gather_rec(const R *__restrict__ in, const uint32_t *__restrict__ perm,
                             uint32_t n, R *__restrict__ out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[perm[i]];
}

void launch_gather_boxes(const Box *in, const uint32_t *perm, uint32_t n, Box *out,
                         hipStream_t st)
{
    if (n) k_gather_rec<Box><<<(n + kBlock - 1) / kBlock, kBlock, 0, st>>>(in, perm, n, out);
}

void launch_gather_aligns(const Align *in, const uint32_t *perm, uint32_t n, Align *out,
                          hipStream_t st)
{
    if (n) k_gather_rec<Align><<<(n + kBlock - 1) / kBlock, kBlock, 0, st>>>(in, perm, n, out);
}

// ------------------------------------------------------------------ per-query LDS sorts
// The runs of one query are contiguous, so the record sorts of merging, selection
// and reporting are segmented sorts: one block per query sorts its records in LDS
// with a bitonic network on indices.  Ties between equal records fall back to the
// input position, which makes the order total and the result deterministic.
// Segments longer than kSegCap go through the global radix sort instead.
// MODE 0: merge order (s, qs, ds, qe, de); MODE 1: selection order (kept boxes
// first, then length descending, s, qs, ds, qe, de).  Length = min of the spans.
template <int MODE>
struct BoxLess {
    __device__ bool operator()(const Box &x, const Box &y) const
    {
        if (MODE == 1) {
            const bool vx = x.q >= 0, vy = y.q >= 0;
            if (vx != vy) return vx;
            if (!vx) return false;
            const int32_t lx = min(x.qe - x.qs, x.de - x.ds), ly = min(y.qe - y.qs, y.de - y.ds);
            if (lx != ly) return lx > ly;
        }
        if (x.s != y.s) return x.s < y.s;
        if (x.qs != y.qs) return x.qs < y.qs;
        if (x.ds != y.ds) return x.ds < y.ds;
        if (x.qe != y.qe) return x.qe < y.qe;
        return x.de < y.de;
    }
};

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_seg_sort_box(const Box *__restrict__ in,
                                                         Box *__restrict__ out,
                                                         const uint32_t *__restrict__ seg_off)
{
    __shared__ Box s_r[kSegCap];
    __shared__ uint16_t s_ix[kSegCap];
    const uint32_t a0 = seg_off[blockIdx.x], n = seg_off[blockIdx.x + 1] - a0;
    if (n == 0 || n > (uint32_t)kSegCap) return;  // longer segments take the global sort
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) s_r[i] = in[a0 + i];
    lds_bitonic(s_r, s_ix, n, BoxLess<MODE>());
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) out[a0 + i] = s_r[s_ix[i]];
}

void launch_seg_sort_box(int mode, const Box *in, Box *out, const uint32_t *seg_off, int32_t nq,
                         hipStream_t st)
{
    if (nq <= 0) return;
    if (mode == 0) k_seg_sort_box<0><<<nq, kBlock, 0, st>>>(in, out, seg_off);
    else k_seg_sort_box<1><<<nq, kBlock, 0, st>>>(in, out, seg_off);
}

// A replayed wave's merge and selection order for one query in one block: its
// boxes sorted by merge order (s, qs, ds, qe, de) in LDS and put in that order,
// each sequence's group swept in place as k_merge_sweep does (merged boxes from
// the group's start, the rest marked empty), then sorted by selection order and
// written out.  The same three steps as k_seg_sort_box<0>, k_merge_sweep and
// k_seg_sort_box<1>, with the boxes kept in LDS between them.
__global__ __launch_bounds__(kBlock) void k_merge_select_seg(const Box *__restrict__ in,
                                                             Box *__restrict__ out,
                                                             const uint32_t *__restrict__ seg_off,
                                                             WaveCtl *__restrict__ ctl)
{
    __shared__ Box s_r[kSegCap];
    __shared__ uint16_t s_ix[kSegCap];
    if ((int32_t)blockIdx.x >= ctl->nqw) return;
    const uint32_t a0 = seg_off[blockIdx.x], n = seg_off[blockIdx.x + 1] - a0;
    if (n > (uint32_t)kSegCap) {
        if (threadIdx.x == 0) ctl->qflag[ctl->qa + (int32_t)blockIdx.x] = 1u;
        return;
    }
    if (n == 0) return;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) s_r[i] = in[a0 + i];
    lds_bitonic(s_r, s_ix, n, BoxLess<0>());  // starts and ends with a barrier
    constexpr int kPer = kSegCap / kBlock;
    Box tmp[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const uint32_t i = threadIdx.x + k * kBlock;
        if (i < n) tmp[k] = s_r[s_ix[i]];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const uint32_t i = threadIdx.x + k * kBlock;
        if (i < n) s_r[i] = tmp[k];
    }
    __syncthreads();
    // the thread at each group's first box sweeps it; a group's first slot always
    // keeps a box of that sequence, so a neighbour's end test reads a valid s
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        if (i > 0 && s_r[i - 1].s == s_r[i].s) continue;
        Box cur = s_r[i];
        const int32_t sq = cur.s;
        uint32_t w = i, j = i + 1;
        for (; j < n; ++j) {
            const Box h = s_r[j];
            if (h.s != sq) break;
            if (h.qs < cur.qe && h.ds < cur.de && cur.ds < h.de) {
                cur.qs = min(cur.qs, h.qs);
                cur.qe = max(cur.qe, h.qe);
                cur.ds = min(cur.ds, h.ds);
                cur.de = max(cur.de, h.de);
                cur.dmin = min(cur.dmin, h.dmin);
                cur.dmax = max(cur.dmax, h.dmax);
            } else {
                s_r[w++] = cur;
                cur = h;
            }
        }
        s_r[w++] = cur;
        for (; w < j; ++w) s_r[w].q = -1;
    }
    __syncthreads();
    lds_bitonic(s_r, s_ix, n, BoxLess<1>());
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) out[a0 + i] = s_r[s_ix[i]];
}

void launch_merge_select_seg(const Box *in, Box *out, const uint32_t *seg_off, int32_t nq_cap,
                             WaveCtl *ctl, hipStream_t st)
{
    if (nq_cap > 0) k_merge_select_seg<<<nq_cap, kBlock, 0, st>>>(in, out, seg_off, ctl);
}

// Report order: alignments with score > 0 first, score descending, then seq,
// q_start, d_start, q_end, d_end and the box.
struct AlignLess {
    __device__ bool operator()(const Align &x, const Align &y) const
    {
        const bool vx = x.score > 0, vy = y.score > 0;
        if (vx != vy) return vx;
        if (!vx) return false;
        if (x.score != y.score) return x.score > y.score;
        if (x.seq_id != y.seq_id) return x.seq_id < y.seq_id;
        if (x.q_start != y.q_start) return x.q_start < y.q_start;
        if (x.d_start != y.d_start) return x.d_start < y.d_start;
        if (x.q_end != y.q_end) return x.q_end < y.q_end;
        if (x.d_end != y.d_end) return x.d_end < y.d_end;
        if (x.box_q_start != y.box_q_start) return x.box_q_start < y.box_q_start;
        if (x.box_d_start != y.box_d_start) return x.box_d_start < y.box_d_start;
        if (x.box_q_end != y.box_q_end) return x.box_q_end < y.box_q_end;
        if (x.box_d_end != y.box_d_end) return x.box_d_end < y.box_d_end;
        return x.band_d0 < y.band_d0;
    }
};

// One block per query: sort its aligned boxes, record the range of those with
// score > 0, and (device form) write the first cap of them as gg_hit records.
__global__ __launch_bounds__(kBlock) void k_report_seg(const Align *__restrict__ in,
                                                       Align *__restrict__ out,
                                                       const uint32_t *__restrict__ sel_off,
                                                       uint32_t *__restrict__ rstart,
                                                       uint32_t *__restrict__ rend, int32_t qa,
                                                       int32_t cap, int32_t *__restrict__ dev_out,
                                                       int32_t *__restrict__ dev_n,
                                                       WaveCtl *__restrict__ ctl)
{
    __shared__ Align s_r[kSegCap];
    __shared__ uint16_t s_ix[kSegCap];
    __shared__ uint32_t s_valid;
    const int32_t ql = blockIdx.x;
    if (ctl) {
        if (ql >= ctl->nqw) return;
        qa = ctl->qa;
    }
    const uint32_t a0 = sel_off[ql], n = sel_off[ql + 1] - a0;
    if (ctl && n > (uint32_t)kSegCap && threadIdx.x == 0) ctl->qflag[qa + ql] = 1u;
    if (n > (uint32_t)kSegCap) return;  // longer segments take the global sort
    if (threadIdx.x == 0) s_valid = 0;
    __syncthreads();
    uint32_t v = 0;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        s_r[i] = in[a0 + i];
        v += s_r[i].score > 0 ? 1u : 0u;
    }
    if (v) atomicAdd(&s_valid, v);
    lds_bitonic(s_r, s_ix, n, AlignLess());  // starts and ends with a barrier
    const uint32_t nv = s_valid;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) out[a0 + i] = s_r[s_ix[i]];
    if (threadIdx.x == 0) {
        rstart[ql] = a0;
        rend[ql] = a0 + nv;
        if (dev_n) dev_n[qa + ql] = (int32_t)nv;
    }
    if (dev_out) {
        const uint32_t m = min(nv, (uint32_t)cap);
        int32_t *dst = dev_out + ((size_t)(qa + ql) * (size_t)cap) * kHitInts;
        for (uint32_t e = threadIdx.x; e < m * kHitInts; e += blockDim.x) {
            const int32_t *src = reinterpret_cast<const int32_t *>(&s_r[s_ix[e / kHitInts]]);
            dst[e] = src[1 + e % kHitInts];
        }
    }
}

void launch_report_seg(const Align *in, Align *out, const uint32_t *sel_off, int32_t nq,
                       uint32_t *rstart, uint32_t *rend, int32_t qa, int32_t cap, int32_t *dev_out,
                       int32_t *dev_n, hipStream_t st, WaveCtl *ctl)
{
    if (nq > 0)
        k_report_seg<<<nq, kBlock, 0, st>>>(in, out, sel_off, rstart, rend, qa, cap, dev_out, dev_n,
                                            ctl);
}

// ------------------------------------------------------------------ S7: merge overlaps
// Boxes sorted by (q, s, qs, ds, qe, de).  Each (q, s) group is swept once by one
// thread, merging the next box into the open one when both their query and
// data-bank intervals intersect; the merged boxes are written from the group's
// start and its remaining slots are marked empty (q = -1).  Each thread owns a
// chunk of `chunk` consecutive boxes (up to kSweepChunk, fewer when there are few
// boxes, down to one per thread) and sweeps every group that starts in it (a group
// may run on past the chunk), so all lanes have work however the groups fall; the
// boxes before the chunk's first group start belong to an earlier chunk's group.
constexpr uint32_t kSweepChunk = 32;

__global__ void k_merge_sweep(const Box *__restrict__ s, uint32_t n, Box *__restrict__ out,
                              uint32_t chunk)
{
    const uint32_t nchunk = (n + chunk - 1) / chunk;
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < nchunk;
         c += gridDim.x * blockDim.x) {
    const uint32_t lo = c * chunk, hi = min(lo + chunk, n);
    uint32_t i = lo;
    if (i > 0) {
        const Box p = s[i - 1];
        while (i < hi) {
            const Box b = s[i];
            if (b.q != p.q || b.s != p.s) break;
            ++i;
        }
    }
    while (i < hi) {  // i starts a group
    const Box first = s[i];
    Box cur = first;
    uint32_t w = i, j = i + 1;
    bool open = true;
    while (open && j < n) {
        // four boxes loaded together, so a long group's walk waits on one load in four
        constexpr uint32_t kAhead = 4;
        Box h[kAhead];
#pragma unroll
        for (uint32_t x = 0; x < kAhead; ++x)
            if (j + x < n) h[x] = s[j + x];
#pragma unroll
        for (uint32_t x = 0; x < kAhead; ++x) {
            if (!open || j >= n) break;
            if (h[x].q != first.q || h[x].s != first.s) {
                open = false;
                break;
            }
            if (h[x].qs < cur.qe && h[x].ds < cur.de && cur.ds < h[x].de) {
                cur.qs = min(cur.qs, h[x].qs);
                cur.qe = max(cur.qe, h[x].qe);
                cur.ds = min(cur.ds, h[x].ds);
                cur.de = max(cur.de, h[x].de);
                cur.dmin = min(cur.dmin, h[x].dmin);
                cur.dmax = max(cur.dmax, h[x].dmax);
            } else {
                out[w++] = cur;
                cur = h[x];
            }
            ++j;
        }
    }
    out[w++] = cur;
    for (; w < j; ++w) out[w].q = -1;
    i = j;  // the next group starts where this one ended
    }
    }
}

// S7 in windows of whole groups.  Boxes leave the extension grouped by (query,
// sequence), and a merge only ever joins boxes of one group, so each group can be
// ordered by (qs, ds, qe, de) and swept on its own.  Block b owns the groups that
// start in positions [b W, b W + W) (W = kMergeWin); a group of at most W boxes
// ends before b W + 2 W, so the block holds all its boxes.  Each box of an owned
// group becomes one 64-bit key (group rank | qs | d + bias | qe): the boxes leave
// the extension unmerged, so ds = qs + d and de = qe + d, and the key orders a
// group exactly as (qs, ds, qe, de) does (equal keys are equal boxes).  The keys
// are sorted in LDS (radix passes) and the owned groups are then swept from their
// keys with the result of k_merge_sweep's one-thread sweep, in parallel over the
// window (merge_sweep_parallel) or, when that has not settled, one thread per
// group: merged boxes from the group's first position, the rest marked empty.  A group that may not fit (the last one the
// block owns, when no other group starts before the block's reach) is recorded
// in big[1 ..] as (first, end) and left to the global sort; big[0] counts them.
constexpr uint32_t kMergeWin = 1024;
constexpr uint32_t kMergeSpan = 2 * kMergeWin;

// Stable LSD radix sort of the m <= kMergeSpan keys in s_key (LDS), 8 bits per
// pass, by a 256-thread block.  Wave w holds keys [512 w, 512 w + 512) in
// registers, 64 per round; a key's rank among equal digits of its wave comes from
// eight ballots (as the global passes rank a tile), the block scans the per-wave
// digit counts, and the keys are written to their places in s_key and read back
// for the next pass.  Only passes whose digit varies across the keys run
// (`varying`: OR of every key XOR the first), digits from bit `lo` up (keys equal
// from bit lo up keep their order).
__device__ void lds_radix_sort(uint64_t *__restrict__ s_key, uint32_t m, uint64_t varying, int lo)
{
    constexpr int kPerWave = kMergeSpan / (kBlock / 64);  // 512
    constexpr int kRounds = kPerWave / 64;                 // 8
    __shared__ uint16_t s_wc[kBlock / 64][kRadix];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t below = (1ull << lane) - 1ull;
    uint64_t k[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const uint32_t idx = w * kPerWave + r * 64 + lane;
        k[r] = idx < m ? s_key[idx] : 0ull;
    }
    for (int shift = lo; shift < 64; shift += kRadixBits) {
        if (((varying >> shift) & (kRadix - 1)) == 0) continue;  // same digit everywhere
#pragma unroll
        for (int i = 0; i < kBlock / 64; ++i) s_wc[i][threadIdx.x] = 0;
        __syncthreads();
        uint32_t rank[kRounds];
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
            const uint32_t idx = w * kPerWave + r * 64 + lane;
            const bool ok = idx < m;
            const uint32_t d = (uint32_t)(k[r] >> shift) & (kRadix - 1);
            uint64_t peers = __ballot(ok);
            // keys past m read as 0 (digit 0): clear in every bit's ballot
#pragma unroll
            for (int b = 0; b < kRadixBits; ++b) {
                const int32_t mk = (int32_t)(d << (31 - b)) >> 31;  // all ones when bit b is set
                const uint64_t bb = __ballot(mk != 0);
                peers &= ~(bb ^ (((uint64_t)(uint32_t)mk << 32) | (uint32_t)mk));
            }
            const uint32_t before = s_wc[w][d];
            rank[r] = before + (uint32_t)__popcll(peers & below);
            __builtin_amdgcn_wave_barrier();
            if (ok && (peers & below) == 0) s_wc[w][d] = (uint16_t)(before + (uint32_t)__popcll(peers));
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        {
            const uint32_t d = threadIdx.x;
            uint32_t run = 0, wc[kBlock / 64];
#pragma unroll
            for (int i = 0; i < kBlock / 64; ++i) {
                wc[i] = run;
                run += s_wc[i][d];
            }
            uint32_t tot;
            const uint32_t start = block_excl_scan<uint32_t>(run, &tot);
#pragma unroll
            for (int i = 0; i < kBlock / 64; ++i) s_wc[i][d] = (uint16_t)(start + wc[i]);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
            const uint32_t idx = w * kPerWave + r * 64 + lane;
            if (idx < m) {
                const uint32_t d = (uint32_t)(k[r] >> shift) & (kRadix - 1);
                s_key[s_wc[w][d] + rank[r]] = k[r];
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
            const uint32_t idx = w * kPerWave + r * 64 + lane;
            if (idx < m) k[r] = s_key[idx];
        }
    }
    __syncthreads();
}

// Orders each run of the m keys in s_key that are equal from bit lo up by the
// whole key, after a sort that left such runs in their input order: odd-even
// transposition rounds over adjacent keys of one run, until a round swaps none
// (true) or `rounds` rounds have passed (false; the runs may be out of order).
// Runs are short (boxes that start on one diagonal at one query position), so
// one round that swaps nothing is the usual cost.
constexpr int kTieRounds = 8;

__device__ bool lds_order_ties(uint64_t *__restrict__ s_key, uint32_t m, int lo, int rounds)
{
    for (int round = 0; round < rounds; ++round) {
        bool swapped = false;
#pragma unroll
        for (int phase = 0; phase < 2; ++phase) {
            for (uint32_t i = 2 * threadIdx.x + phase; i + 1 < m; i += 2 * kBlock) {
                const uint64_t a = s_key[i], b = s_key[i + 1];
                if ((a >> lo) == (b >> lo) && a > b) {
                    s_key[i] = b;
                    s_key[i + 1] = a;
                    swapped = true;
                }
            }
            __syncthreads();
        }
        if (!__syncthreads_or(swapped)) return true;
    }
    return false;
}

// Length bin of a box for the selection prefilter (length >> shift, clamped) and
// its slot record (q << 10) | bin.
__device__ __forceinline__ uint32_t len_bin(const Box &b, int shift)
{
    return min((uint32_t)min(b.qe - b.qs, b.de - b.ds) >> shift, (uint32_t)(kLenBins - 1));
}

__device__ __forceinline__ uint32_t len_record(const Box &b, int shift)
{
    return ((uint32_t)b.q << 10) | len_bin(b, shift);
}

static_assert(kLenBins == 1024, "length records keep the bin in 10 bits");

// The running union of a sweep's merged boxes: query start, end, bank start, end,
// extreme diagonals.
struct MAgg {
    int32_t qs, qe, ds, de, dmin, dmax;
};

__device__ __forceinline__ MAgg magg_none()
{
    return MAgg{INT32_MAX, INT32_MIN, INT32_MAX, INT32_MIN, INT32_MAX, INT32_MIN};
}

__device__ __forceinline__ MAgg magg_join(const MAgg &a, const MAgg &b)
{
    return MAgg{min(a.qs, b.qs), max(a.qe, b.qe), min(a.ds, b.ds),
                max(a.de, b.de), min(a.dmin, b.dmin), max(a.dmax, b.dmax)};
}

// The sweep's test: box (qs, ds, de) joins the running union cur.
__device__ __forceinline__ bool magg_takes(const MAgg &cur, int32_t qs, int32_t ds, int32_t de)
{
    return qs < cur.qe && ds < cur.de && cur.ds < de;
}

__device__ __forceinline__ MAgg magg_shfl_up(const MAgg &a, int o)
{
    return MAgg{__shfl_up(a.qs, o, 64), __shfl_up(a.qe, o, 64), __shfl_up(a.ds, o, 64),
                __shfl_up(a.de, o, 64), __shfl_up(a.dmin, o, 64), __shfl_up(a.dmax, o, 64)};
}

// Exclusive segmented scan over the block's threads: thread t holds (f, a) = (a
// segment starts in its items, union of its items from its last start on); it
// receives the union over the items before its own back to the last start (the
// union of the segment its first item continues).  Pairs combine as (f1, a1) then
// (f2, a2) -> (f1 | f2, f2 ? a2 : a1 + a2).
__device__ MAgg seg_excl_union(bool f, const MAgg &a, bool *start_before = nullptr)
{
    __shared__ int32_t s_wf[kBlock / 64];
    __shared__ MAgg s_wa[kBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int32_t fi = f ? 1 : 0;
    MAgg x = a;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t yf = __shfl_up(fi, o, 64);
        const MAgg y = magg_shfl_up(x, o);
        if (lane >= o) {
            if (!fi) x = magg_join(y, x);
            fi |= yf;
        }
    }
    if (lane == 63) {
        s_wf[w] = fi;
        s_wa[w] = x;
    }
    int32_t ef = __shfl_up(fi, 1, 64);
    MAgg ex = magg_shfl_up(x, 1);
    if (lane == 0) {
        ef = 0;
        ex = magg_none();
    }
    __syncthreads();
    MAgg pre = magg_none();
    int32_t pf = 0;
    for (int i = 0; i < w; ++i) {
        pre = s_wf[i] ? s_wa[i] : magg_join(pre, s_wa[i]);
        pf |= s_wf[i];
    }
    __syncthreads();  // s_wf and s_wa are rewritten by the next call
    if (start_before) *start_before = (ef | pf) != 0;
    return ef ? ex : magg_join(pre, ex);
}

// Parallel form of the sweep of a window's owned groups (keys [0, m) sorted in
// s_key, group g's keys [s_start[g] - o, s_start[g + 1] - o)).  Thread t takes keys
// [8 t, 8 t + 8).  A key starts a merged box when it starts its group or the sweep
// does not join it to the union before it.  Tentative starts: group starts and
// the keys that do not join the one box before them (a box that joins its
// predecessor joins any union holding it).  Each round scans the unions of the
// tentative segments and drops the starts that join the union before them; the
// test only gets easier as unions grow, and tentative segments are never larger
// than the sweep's, so a dropped start is never a start of the sweep, and when a
// round drops nothing every key's union is the sweep's and the starts are
// exactly its.  Returns false (nothing written) when `rounds` rounds did not
// settle; the caller then sweeps group by group.
__device__ bool merge_sweep_parallel(const uint64_t *__restrict__ s_key, uint32_t m,
                                     const uint16_t *__restrict__ s_start, uint32_t o,
                                     uint32_t nw, uint16_t *__restrict__ s_pg,
                                     uint8_t *__restrict__ s_f8, int bl, int bd, int32_t bias,
                                     const Box *__restrict__ in, Box *__restrict__ out,
                                     uint32_t at, int rounds, LenSel ls)
{
    constexpr int kPer = kMergeSpan / kBlock;  // 8 keys per thread
    const uint64_t mbl = (1ull << bl) - 1ull, mbd = (1ull << bd) - 1ull;
    const int gsh = 2 * bl + bd;
    const uint32_t j0 = threadIdx.x * kPer;
    // key j's box (read from LDS on each pass rather than held in registers)
    auto box_of = [&](uint64_t key) {
        const int32_t qe = (int32_t)(key & mbl);
        const int32_t d = (int32_t)((key >> bl) & mbd) - bias;
        const int32_t qs = (int32_t)((key >> (bl + bd)) & mbl);
        return MAgg{qs, qe, qs + d, qe + d, d, d};
    };
    uint32_t V = 0, F = 0, GS = 0;  // valid keys, tentative starts, group starts
    {
        uint64_t prev = j0 > 0 && j0 < m ? s_key[j0 - 1] : 0ull;
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const uint32_t j = j0 + r;
            if (j >= m) break;
            const uint64_t key = s_key[j];
            const bool gs = j == 0 || (prev >> gsh) != (key >> gsh);
            bool st = gs;
            if (!gs) {
                const MAgg a = box_of(prev), b = box_of(key);
                st = !magg_takes(a, b.qs, b.ds, b.de);
            }
            V |= 1u << r;
            if (gs) GS |= 1u << r;
            if (st) F |= 1u << r;
            prev = key;
        }
    }
    MAgg carry;
    for (int round = 0;; ++round) {
        if (round == rounds) return false;
        bool sf = false;
        MAgg sa = magg_none();
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            if (!((V >> r) & 1u)) continue;
            const MAgg b = box_of(s_key[j0 + r]);
            if ((F >> r) & 1u) {
                sf = true;
                sa = b;
            } else {
                sa = magg_join(sa, b);
            }
        }
        carry = seg_excl_union(sf, sa);
        MAgg run = carry;
        bool changed = false;
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            if (!((V >> r) & 1u)) continue;
            const uint32_t bit = 1u << r;
            const MAgg b = box_of(s_key[j0 + r]);
            if ((F & bit) && !(GS & bit) && magg_takes(run, b.qs, b.ds, b.de)) {
                F &= ~bit;
                changed = true;
            }
            run = (F & bit) ? b : magg_join(run, b);
        }
        if (!__syncthreads_or(changed)) break;
    }
    // merged box k of group g goes to the group's k-th position: k is its rank
    // among the group's starts, P(j) - P(first key of g) with P(j) the starts in
    // [0, j]; the group's remaining positions are marked empty
    uint32_t tot;
    const uint32_t before = block_excl_scan<uint32_t>((uint32_t)__popc(F), &tot);
    s_f8[threadIdx.x] = (uint8_t)F;
#pragma unroll
    for (int r = 0; r < kPer; ++r)
        if ((GS >> r) & 1u)
            s_pg[(uint32_t)(s_key[j0 + r] >> gsh)] = (uint16_t)(before + __popc(F & ((2u << r) - 1u)));
    __syncthreads();
    MAgg run = carry;
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        if (!((V >> r) & 1u)) continue;
        const uint32_t j = j0 + r;
        const uint64_t key = s_key[j];
        const uint32_t g = (uint32_t)(key >> gsh);
        const MAgg b = box_of(key);
        run = ((F >> r) & 1u) ? b : magg_join(run, b);
        const uint32_t first = (uint32_t)s_start[g] - o;
        const uint32_t p0 = s_pg[g];
        const uint32_t nseg = (g + 1 < nw ? (uint32_t)s_pg[g + 1] - 1u : tot) - p0 + 1u;
        if (j - first >= nseg) {
            out[at + j].q = -1;
            if (ls.binq) ls.binq[at + j] = kNoBin;
        }
        const bool last = j + 1 >= m || (r + 1 < kPer ? ((F >> (r + 1)) & 1u) != 0
                                                        : (s_f8[threadIdx.x + 1] & 1u) != 0);
        if (!last) continue;
        const uint32_t rank = before + __popc(F & ((2u << r) - 1u)) - p0;
        const int2 qsid = *reinterpret_cast<const int2 *>(in + at + j);
        const Box bx{qsid.x, qsid.y, run.qs, run.qe, run.ds, run.de, run.dmin, run.dmax};
        out[at + first + rank] = bx;
        if (ls.binq) ls.binq[at + first + rank] = len_record(bx, ls.shift);
    }
    return true;
}

__global__ __launch_bounds__(kBlock, 6) void k_merge_tiles(const Box *__restrict__ in, uint32_t n,
                                                        int bl, int bd, int32_t bias,
                                                        Box *__restrict__ out,
                                                        uint32_t *__restrict__ big, uint32_t big_cap,
                                                        int rounds, LenSel ls)
{
    __shared__ uint64_t s_key[kMergeSpan];
    __shared__ uint16_t s_start[kMergeSpan + 1];
    __shared__ uint16_t s_rank[kMergeSpan];
    __shared__ uint32_t s_wc[kBlock / 64];
    __shared__ uint32_t s_nw;
    __shared__ uint64_t s_vary[2];
    const uint32_t base = blockIdx.x * kMergeWin;
    if (base >= n) return;
    if (threadIdx.x == 0) s_vary[0] = s_vary[1] = 0;
    const uint32_t lim = min(base + kMergeSpan, n);
    const uint32_t R = lim - base;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t below = (1ull << lane) - 1ull;
    // group starts in [base, lim), in order, and each position's group rank; past
    // the window's first kMergeWin positions only up to the first start found (it
    // ends the last owned group)
    uint32_t ns = 0, nwin = 0;
    for (uint32_t u = 0; u < kMergeSpan / kBlock; ++u) {
        const uint32_t r = u * kBlock + threadIdx.x;
        const uint32_t p = base + r;
        int2 a = make_int2(-1, -1);
        if (r < R) a = *reinterpret_cast<const int2 *>(in + p);
        // the position before: the lane below holds it; lane 0 reads it
        int2 b = make_int2(__shfl_up(a.x, 1, 64), __shfl_up(a.y, 1, 64));
        if (lane == 0 && r < R && p > 0) b = *reinterpret_cast<const int2 *>(in + p - 1);
        const bool f = r < R && (p == 0 || a.x != b.x || a.y != b.y);
        const uint64_t m = __ballot(f);
        if (lane == 0) s_wc[wv] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t before = ns, round = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) {
            if (w < wv) before += s_wc[w];
            round += s_wc[w];
        }
        const uint32_t at = before + (uint32_t)__popcll(m & below);
        if (f) s_start[at] = (uint16_t)r;
        // rank of r's group among the range's starts (positions before the first
        // start belong to an earlier block's group and are never used)
        if (r < R) s_rank[r] = (uint16_t)(at + (f ? 1u : 0u) - 1u);
        ns += round;
        if (u < kMergeWin / kBlock) nwin = ns;  // starts below kMergeWin
        __syncthreads();
        if (u + 1 >= kMergeWin / kBlock && ns > nwin) break;
    }
    if (threadIdx.x == 0) {
        s_start[ns] = (uint16_t)R;
        uint32_t nw = 0;  // owned groups: starts below kMergeWin
        while (nw < ns && s_start[nw] < kMergeWin) ++nw;
        s_nw = nw;
    }
    __syncthreads();
    uint32_t nw = s_nw;
    if (nw == 0) return;
    if (nw == ns && lim < n) {
        // the last owned group reaches past the range: find its end, leave it to
        // the global sort
        const uint32_t p0 = base + s_start[nw - 1];
        if (wv == 0) {
            const int2 g = *reinterpret_cast<const int2 *>(in + p0);
            uint32_t end = n;
            for (uint32_t p = lim; p < n; p += 64) {
                const uint32_t pp = p + lane;
                bool other = false;
                if (pp < n) {
                    const int2 a = *reinterpret_cast<const int2 *>(in + pp);
                    other = a.x != g.x || a.y != g.y;
                }
                const uint64_t m = __ballot(other);
                if (m) {
                    end = p + (uint32_t)__ffsll((unsigned long long)m) - 1;
                    break;
                }
            }
            if (lane == 0) {
                const uint32_t slot = atomicAdd(big, 1u);
                if (slot < big_cap) {
                    big[1 + 2 * slot] = p0;
                    big[2 + 2 * slot] = end;
                }
            }
        }
        --nw;
    }
    if (nw == 0) return;
    const uint32_t o = s_start[0], m = s_start[nw] - o;  // keys of the owned small groups
    const uint64_t mbl = (1ull << bl) - 1ull, mbd = (1ull << bd) - 1ull;
    uint64_t vary = 0, zeros = 0;
    for (uint32_t j = threadIdx.x; j < m; j += kBlock) {
        const Box b = in[base + o + j];
        const uint64_t rank = (uint64_t)(s_rank[o + j] - s_rank[o]);
        const uint64_t d = (uint64_t)(uint32_t)(b.ds - b.qs + bias);
        const uint64_t key = (rank << (2 * bl + bd)) | ((uint64_t)(uint32_t)b.qs << (bl + bd)) |
                             ((d & mbd) << bl) | ((uint64_t)(uint32_t)b.qe & mbl);
        s_key[j] = key;
        vary |= key;
        zeros |= ~key;
    }
    // bits that differ between keys: set in some key and clear in some key
    for (int off = 32; off > 0; off >>= 1) {
        vary |= __shfl_xor(vary, off, 64);
        zeros |= __shfl_xor(zeros, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicOr(reinterpret_cast<unsigned long long *>(&s_vary[0]), (unsigned long long)vary);
        atomicOr(reinterpret_cast<unsigned long long *>(&s_vary[1]), (unsigned long long)zeros);
    }
    __syncthreads();
    // sorted by (rank, qs, d) in passes over the bits above qe; keys equal there
    // (one start on one diagonal) are then put in qe order, or, when there are
    // too many of them, the keys are sorted again over every bit
    lds_radix_sort(s_key, m, s_vary[0] & s_vary[1], bl);
    if (!lds_order_ties(s_key, m, bl, kTieRounds)) lds_radix_sort(s_key, m, s_vary[0] & s_vary[1], 0);
    // the key-building ranks are no longer needed: their space holds the
    // parallel sweep's per-group counts
    if (merge_sweep_parallel(s_key, m, s_start, o, nw, s_rank,
                             reinterpret_cast<uint8_t *>(s_rank + kMergeWin), bl, bd, bias, in, out,
                             base + o, rounds, ls))
        return;
    // sweep each owned group from its keys
    for (uint32_t g = threadIdx.x; g < nw; g += kBlock) {
        const uint32_t j0 = s_start[g] - o, j1 = s_start[g + 1] - o;
        const int2 qsid = *reinterpret_cast<const int2 *>(in + base + o + j0);
        auto decode = [&](uint64_t key) {
            const int32_t qe = (int32_t)(key & mbl);
            const int32_t d = (int32_t)((key >> bl) & mbd) - bias;
            const int32_t qs = (int32_t)((key >> (bl + bd)) & mbl);
            return Box{qsid.x, qsid.y, qs, qe, qs + d, qe + d, d, d};
        };
        // a merged box to its slot, with its length record
        auto emit = [&](uint32_t slot, const Box &bx) {
            out[base + o + slot] = bx;
            if (ls.binq) ls.binq[base + o + slot] = len_record(bx, ls.shift);
        };
        Box cur = decode(s_key[j0]);
        uint32_t w = j0;
        // keys read eight at a time ahead of the fold, which is serial in the group
        constexpr uint32_t kAheadKeys = 8;
        for (uint32_t j = j0 + 1; j < j1; j += kAheadKeys) {
            uint64_t hk[kAheadKeys];
#pragma unroll
            for (uint32_t x = 0; x < kAheadKeys; ++x) hk[x] = s_key[min(j + x, j1 - 1)];
#pragma unroll
            for (uint32_t x = 0; x < kAheadKeys; ++x) {
                if (j + x >= j1) break;
                const Box h = decode(hk[x]);
                if (h.qs < cur.qe && h.ds < cur.de && cur.ds < h.de) {
                    cur.qs = min(cur.qs, h.qs);
                    cur.qe = max(cur.qe, h.qe);
                    cur.ds = min(cur.ds, h.ds);
                    cur.de = max(cur.de, h.de);
                    cur.dmin = min(cur.dmin, h.dmin);
                    cur.dmax = max(cur.dmax, h.dmax);
                } else {
                    emit(w++, cur);
                    cur = h;
                }
            }
        }
        emit(w++, cur);
        for (; w < j1; ++w) {
            out[base + o + w].q = -1;
            if (ls.binq) ls.binq[base + o + w] = kNoBin;
        }
    }
}

// Copy the boxes of nr ranges [ranges[2r], ranges[2r + 1]) between their place
// in `pos` and a packed array (to_packed: pos -> packed at offs[r]; else back).
__global__ void k_copy_ranges(const Box *__restrict__ src, Box *__restrict__ dst,
                              const uint32_t *__restrict__ ranges, const uint32_t *__restrict__ offs,
                              uint32_t nr, int to_packed)
{
    for (uint32_t r = blockIdx.x; r < nr; r += gridDim.x) {
        const uint32_t a = ranges[2 * r], b = ranges[2 * r + 1], o = offs[r];
        for (uint32_t i = threadIdx.x; i < b - a; i += blockDim.x) {
            if (to_packed) dst[o + i] = src[a + i];
            else dst[a + i] = src[o + i];
        }
    }
}

// The sweep of whole groups too big for a window, in parallel: block g takes
// group g, boxes [offs[g], offs[g + 1]) of s (sorted in merge order), in chunks of
// kMergeSpan boxes, eight per thread, as merge_sweep_parallel does a window.  The
// union of the segment still open at a chunk's end is carried into the next
// chunk, where it is the union before every box that no start in the chunk
// precedes.  Merged boxes go to the group's first positions in out, the rest are
// marked empty.  A chunk that has not settled in `rounds` rounds is swept by one
// thread; the results are the same.
__global__ __launch_bounds__(kBlock) void k_merge_groups(const Box *__restrict__ s,
                                                         const uint32_t *__restrict__ offs,
                                                         uint32_t ngroup, Box *__restrict__ out,
                                                         int rounds)
{
    constexpr int kPer = kMergeSpan / kBlock;
    __shared__ MAgg s_open;
    __shared__ uint32_t s_nseg;
    __shared__ uint8_t s_f8[kBlock + 1];
    auto item = [&](uint32_t i) {
        const Box b = s[i];
        return MAgg{b.qs, b.qe, b.ds, b.de, b.dmin, b.dmax};
    };
    for (uint32_t g = blockIdx.x; g < ngroup; g += gridDim.x) {
        const uint32_t a = offs[g], e = offs[g + 1];
        const int2 qsid = *reinterpret_cast<const int2 *>(s + a);
        MAgg open = magg_none();  // union of the segment open before the chunk
        uint32_t nseg = 0;        // merged boxes that start before the chunk
        for (uint32_t c0 = a; c0 < e; c0 += kMergeSpan) {
            const uint32_t m = min((uint32_t)kMergeSpan, e - c0);
            const uint32_t j0 = threadIdx.x * kPer;
            uint32_t V = 0, F = 0;
#pragma unroll
            for (int r = 0; r < kPer; ++r) {
                const uint32_t j = j0 + r;
                if (j >= m) break;
                V |= 1u << r;
                const uint32_t i = c0 + j;
                bool st = i == a;  // the group's first box
                if (!st) {
                    const MAgg p = item(i - 1), b = item(i);
                    st = !magg_takes(p, b.qs, b.ds, b.de);
                }
                if (st) F |= 1u << r;
            }
            const uint32_t GS = (c0 == a && threadIdx.x == 0) ? 1u : 0u;
            MAgg carry = magg_none();
            bool settled = false;
            for (int round = 0; round < rounds; ++round) {
                bool sf = false;
                MAgg sa = magg_none();
#pragma unroll
                for (int r = 0; r < kPer; ++r) {
                    if (!((V >> r) & 1u)) continue;
                    const MAgg b = item(c0 + j0 + r);
                    if ((F >> r) & 1u) {
                        sf = true;
                        sa = b;
                    } else {
                        sa = magg_join(sa, b);
                    }
                }
                bool before = false;
                carry = seg_excl_union(sf, sa, &before);
                if (!before) carry = magg_join(open, carry);
                MAgg run = carry;
                bool changed = false;
#pragma unroll
                for (int r = 0; r < kPer; ++r) {
                    if (!((V >> r) & 1u)) continue;
                    const uint32_t bit = 1u << r;
                    const MAgg b = item(c0 + j0 + r);
                    if ((F & bit) && !(GS & bit) && magg_takes(run, b.qs, b.ds, b.de)) {
                        F &= ~bit;
                        changed = true;
                    }
                    run = (F & bit) ? b : magg_join(run, b);
                }
                if (!__syncthreads_or(changed)) {
                    settled = true;
                    break;
                }
            }
            if (!settled) {
                // one thread sweeps the chunk from the open union
                if (threadIdx.x == 0) {
                    MAgg cur = open;
                    uint32_t k = nseg;
                    for (uint32_t j = 0; j < m; ++j) {
                        const MAgg b = item(c0 + j);
                        if (c0 + j == a) {
                            cur = b;
                            k = 1;
                        } else if (magg_takes(cur, b.qs, b.ds, b.de)) {
                            cur = magg_join(cur, b);
                        } else {
                            out[a + k - 1] = Box{qsid.x, qsid.y, cur.qs, cur.qe, cur.ds, cur.de,
                                                 cur.dmin, cur.dmax};
                            cur = b;
                            ++k;
                        }
                    }
                    if (c0 + m == e)
                        out[a + k - 1] =
                            Box{qsid.x, qsid.y, cur.qs, cur.qe, cur.ds, cur.de, cur.dmin, cur.dmax};
                    s_open = cur;
                    s_nseg = k;
                }
            } else {
                // a segment ends at its last box in the chunk when the next box
                // starts one, or at the group's end; merged box nseg - 1 + P(j), P(j)
                // the chunk's starts up to box j.  The segment open at the chunk's
                // end is carried, and written by the chunk that closes it.
                uint32_t tot;
                const uint32_t pre = block_excl_scan<uint32_t>((uint32_t)__popc(F), &tot);
                s_f8[threadIdx.x] = (uint8_t)F;
                if (threadIdx.x == 0) {
                    s_f8[kBlock] = 0;
                    // a start at the chunk's first box closes the segment carried in
                    if (c0 > a && (F & 1u))
                        out[a + nseg - 1u] = Box{qsid.x, qsid.y, open.qs, open.qe, open.ds, open.de,
                                                 open.dmin, open.dmax};
                }
                __syncthreads();
                MAgg run = carry;
#pragma unroll
                for (int r = 0; r < kPer; ++r) {
                    if (!((V >> r) & 1u)) continue;
                    const uint32_t j = j0 + r;
                    run = ((F >> r) & 1u) ? item(c0 + j) : magg_join(run, item(c0 + j));
                    const uint32_t k = nseg - 1u + pre + (uint32_t)__popc(F & ((2u << r) - 1u));
                    if (j + 1 >= m) {
                        if (c0 + m == e)
                            out[a + k] = Box{qsid.x, qsid.y, run.qs, run.qe, run.ds, run.de,
                                             run.dmin, run.dmax};
                        s_open = run;
                        s_nseg = k + 1u;
                    } else if (r + 1 < kPer ? ((F >> (r + 1)) & 1u) != 0
                                            : (s_f8[threadIdx.x + 1] & 1u) != 0) {
                        out[a + k] = Box{qsid.x, qsid.y, run.qs, run.qe, run.ds, run.de, run.dmin,
                                         run.dmax};
                    }
                }
            }
            __syncthreads();
            open = s_open;
            nseg = s_nseg;
            __syncthreads();  // s_open, s_nseg and s_f8 are rewritten by the next chunk
        }
        for (uint32_t i = a + nseg + threadIdx.x; i < e; i += kBlock) out[i].q = -1;
        __syncthreads();
    }
}

void launch_merge_groups(const Box *sorted, const uint32_t *offs, uint32_t ngroup, Box *out,
                         int rounds, hipStream_t st)
{
    if (ngroup == 0) return;
    k_merge_groups<<<std::min<uint32_t>(ngroup, 65536), kBlock, 0, st>>>(sorted, offs, ngroup, out,
                                                                         rounds);
}

void launch_merge_tiles(const Box *in, uint32_t n, int bl, int bd, int32_t bias, Box *out,
                        uint32_t *big, uint32_t big_cap, int rounds, LenSel ls, hipStream_t st)
{
    if (n == 0) return;
    launch_fill_u32(big, 1, 0u, st);
    const uint32_t nb = (n + kMergeWin - 1) / kMergeWin;
    k_merge_tiles<<<nb, kBlock, 0, st>>>(in, n, bl, bd, bias, out, big, big_cap, rounds, ls);
}

void launch_copy_ranges(const Box *src, Box *dst, const uint32_t *ranges, const uint32_t *offs,
                        uint32_t nr, bool to_packed, hipStream_t st)
{
    if (nr == 0) return;
    k_copy_ranges<<<std::min<uint32_t>(nr, 65536), kBlock, 0, st>>>(src, dst, ranges, offs, nr,
                                                                    to_packed ? 1 : 0);
}

void launch_merge_sweep(const Box *sorted, uint32_t n, Box *out, hipStream_t st)
{
    if (n) {
        // about half a million threads fill the chip; longer chunks only past that
        const uint32_t chunk = std::max<uint32_t>(1, std::min<uint32_t>(kSweepChunk, n >> 19));
        const uint32_t threads = (n + chunk - 1) / chunk;
        k_merge_sweep<<<std::min<uint32_t>((threads + kBlock - 1) / kBlock, kMaxGrid), kBlock, 0,
                        st>>>(sorted, n, out, chunk);
    }
}

// ------------------------------------------------------------------ S8: select
// Records sorted by query first (empty ones last): each query's run [qstart, qend).
__global__ void k_segments_box(const Box *__restrict__ s, uint32_t n, int32_t nq,
                               uint32_t *__restrict__ qstart, uint32_t *__restrict__ qend)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += gridDim.x * blockDim.x) {
        const int32_t q = s[i].q;
        if (q < 0 || q >= nq) continue;
        if (i == 0 || s[i - 1].q != q) qstart[q] = i;
        if (i + 1 == n || s[i + 1].q != q) qend[q] = i + 1;
    }
}

// ------------------------------------------------------------------ S8 prefilter
// Selecting the N longest boxes of a query needs only the boxes at least as long
// as its N-th longest.  A histogram of each query's box lengths (bins of 2^shift,
// kLenBins of them) gives the highest bin whose boxes and the longer ones number
// at least N; every box in or above that bin is kept (a superset of the N longest,
// ties included) and the full order is applied to those alone.  Boxes are in
// query order; empty slots (q < 0) are dropped.

// Length records of n box slots: binq[i] for every slot.
__global__ void k_len_records(const Box *__restrict__ b, uint32_t n, LenSel ls)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int32_t q = b[i].q;
        ls.binq[i] = q >= 0 ? len_record(b[i], ls.shift) : kNoBin;
    }
}

// The same for the slots of nr ranges [ranges[2r], ranges[2r + 1]) (a block per range).
__global__ void k_len_records_ranges(const Box *__restrict__ b, const uint32_t *__restrict__ ranges,
                                     uint32_t nr, LenSel ls)
{
    for (uint32_t r = blockIdx.x; r < nr; r += gridDim.x) {
        const uint32_t a = ranges[2 * r], e = ranges[2 * r + 1];
        for (uint32_t i = a + threadIdx.x; i < e; i += blockDim.x) {
            const int32_t q = b[i].q;
            ls.binq[i] = q >= 0 ? len_record(b[i], ls.shift) : kNoBin;
        }
    }
}

// Per-query length histograms from n slot records: hist[q * kLenBins + bin].  A
// block counts kLenHistTiles tiles of kTile records (thread t reading records
// [8 t, 8 t + 8) of each), so that the blocks of one query add their LDS counts to
// the query's kLenBins counters less often.  Records are in query order: those of
// the block's first query are counted in LDS, any others in global memory.
constexpr int kLenHistTiles = 8;

__global__ __launch_bounds__(kBlock) void k_len_hist(const uint32_t *__restrict__ binq, uint32_t n,
                                                     uint32_t *__restrict__ hist)
{
    __shared__ uint32_t h[kLenBins];
    __shared__ uint32_t s_q0;
    if (threadIdx.x == 0) s_q0 = UINT32_MAX;
    for (int i = threadIdx.x; i < kLenBins; i += kBlock) h[i] = 0;
    const int64_t b0 = (int64_t)blockIdx.x * kLenHistTiles * kTile;
    // the block's first query: the smallest query of its records
    uint32_t q0 = UINT32_MAX;
#pragma unroll 2
    for (int t = 0; t < kLenHistTiles; ++t) {
        uint32_t v[kItems];
        const int64_t i0 = b0 + (int64_t)t * kTile + (int64_t)threadIdx.x * kItems;
        load_items<uint32_t>(binq, i0, n, v);
#pragma unroll
        for (int r = 0; r < kItems; ++r)
            if (i0 + r < (int64_t)n && v[r] != kNoBin) q0 = min(q0, v[r] >> 10);
    }
    __syncthreads();
    if (q0 != UINT32_MAX) atomicMin(&s_q0, q0);
    __syncthreads();
    q0 = s_q0;
#pragma unroll 2
    for (int t = 0; t < kLenHistTiles; ++t) {
        uint32_t v[kItems];
        const int64_t i0 = b0 + (int64_t)t * kTile + (int64_t)threadIdx.x * kItems;
        load_items<uint32_t>(binq, i0, n, v);
#pragma unroll
        for (int r = 0; r < kItems; ++r) {
            if (i0 + r >= (int64_t)n || v[r] == kNoBin) continue;
            const uint32_t bin = v[r] & (kLenBins - 1);
            if ((v[r] >> 10) == q0) atomicAdd(&h[bin], 1u);
            else atomicAdd(&hist[(size_t)(v[r] >> 10) * kLenBins + bin], 1u);
        }
    }
    __syncthreads();
    if (q0 != UINT32_MAX)
        for (int i = threadIdx.x; i < kLenBins; i += kBlock)
            if (h[i]) atomicAdd(&hist[(size_t)q0 * kLenBins + i], h[i]);
}

// One block per query: its box count (all bins) and the highest bin whose boxes
// and the longer ones number at least N (bin 0 when the query has fewer).
__global__ __launch_bounds__(kBlock) void k_len_threshold(const uint32_t *__restrict__ hist,
                                                          int32_t nq, int32_t N,
                                                          uint32_t *__restrict__ thr,
                                                          uint32_t *__restrict__ nvalid)
{
    constexpr int kPer = kLenBins / kBlock;  // bins per thread, highest bins to thread 0
    for (int32_t q = blockIdx.x; q < nq; q += gridDim.x) {
        const uint32_t *h = hist + (size_t)q * kLenBins;
        uint32_t c[kPer], sum = 0;
#pragma unroll
        for (int r = 0; r < kPer; ++r) {  // thread t holds bins from the top: t * kPer + r
            c[r] = h[kLenBins - 1 - (threadIdx.x * kPer + r)];
            sum += c[r];
        }
        uint32_t tot;
        uint32_t above = block_excl_scan<uint32_t>(sum, &tot);  // boxes in higher bins
        uint32_t best = 0;  // a thread that crosses N names the bin; crossing is unique
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const uint32_t before = above;
            above += c[r];
            if (before < (uint32_t)N && above >= (uint32_t)N)
                best = (uint32_t)(kLenBins - 1 - (threadIdx.x * kPer + r)) + 1;  // bin + 1
        }
        uint32_t pick;
        block_excl_scan<uint32_t>(best, &pick);  // sum: at most one thread is non-zero
        if (threadIdx.x == 0) {
            thr[q] = pick ? pick - 1 : 0u;
            nvalid[q] = tot;
        }
    }
}

// Stable compaction of the kept boxes, in two passes over tiles (count; write at
// the scanned tile offsets), so the kept boxes stay in query order.  Both passes
// decide from the slots' length records; only the write pass reads the boxes it
// keeps.
__global__ __launch_bounds__(kBlock) void k_len_keep(const Box *__restrict__ b,
                                                     const uint32_t *__restrict__ binq, uint32_t n,
                                                     const uint32_t *__restrict__ thr,
                                                     const uint32_t *__restrict__ tile_off,
                                                     uint32_t *__restrict__ counts,
                                                     Box *__restrict__ out)
{
    const uint32_t base = blockIdx.x * (uint32_t)kTile;
    uint32_t at = tile_off ? tile_off[blockIdx.x] : 0u, c = 0;
    uint32_t rec[kItems];
    load_items<uint32_t>(binq, (int64_t)base + (int64_t)threadIdx.x * kItems, n, rec);
    // thread t holds slots base + t kItems .. + kItems - 1
    bool keep[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const uint32_t i = base + threadIdx.x * kItems + r;
        keep[r] = i < n && rec[r] != kNoBin && (rec[r] & (kLenBins - 1)) >= thr[rec[r] >> 10];
        c += keep[r] ? 1u : 0u;
    }
    uint32_t tot;
    const uint32_t ex = block_excl_scan<uint32_t>(c, &tot);
    if (!tile_off) {
        if (threadIdx.x == 0) counts[blockIdx.x] = tot;
        return;
    }
    at += ex;
#pragma unroll
    for (int r = 0; r < kItems; ++r)
        if (keep[r]) out[at++] = b[base + threadIdx.x * kItems + r];
}

void launch_len_records(const Box *b, uint32_t n, LenSel ls, hipStream_t st)
{
    if (n == 0) return;
    k_len_records<<<std::min<uint32_t>((n + kBlock - 1) / kBlock, kMaxGrid), kBlock, 0, st>>>(b, n,
                                                                                          ls);
}

void launch_len_records_ranges(const Box *b, const uint32_t *ranges, uint32_t nr, LenSel ls,
                               hipStream_t st)
{
    if (nr == 0) return;
    k_len_records_ranges<<<std::min<uint32_t>(nr, 65536), kBlock, 0, st>>>(b, ranges, nr, ls);
}

void launch_len_prefilter(const uint32_t *binq, uint32_t n, int32_t nq, int32_t N,
                          uint32_t *hist, uint32_t *thr, uint32_t *nvalid,
                          uint32_t *tile_counts, uint32_t *partials, hipStream_t st)
{
    if (n == 0 || nq <= 0) return;
    const uint32_t tiles = (n + kTile - 1) / kTile;
    launch_fill_u32(hist, (size_t)nq * kLenBins, 0u, st);
    k_len_hist<<<(tiles + kLenHistTiles - 1) / kLenHistTiles, kBlock, 0, st>>>(binq, n, hist);
    k_len_threshold<<<std::min<uint32_t>((uint32_t)nq, kMaxGrid), kBlock, 0, st>>>(hist, nq, N, thr,
                                                                                   nvalid);
    k_len_keep<<<tiles, kBlock, 0, st>>>(nullptr, binq, n, thr, nullptr, tile_counts, nullptr);
    launch_scan_u32(tile_counts, tile_counts, tiles, partials, st);  // kept total at [tiles]
}

void launch_len_compact(const Box *b, const uint32_t *binq, uint32_t n, const uint32_t *thr,
                        const uint32_t *tile_off, Box *out, hipStream_t st)
{
    if (n == 0) return;
    k_len_keep<<<(n + kTile - 1) / kTile, kBlock, 0, st>>>(b, binq, n, thr, tile_off, nullptr, out);
}

void launch_segments_box(const Box *sorted, uint32_t n, int32_t nq, uint32_t *qstart,
                         uint32_t *qend, hipStream_t st)
{
    if (n)
        k_segments_box<<<std::min<uint32_t>((n + kBlock - 1) / kBlock, kMaxGrid), kBlock, 0, st>>>(
            sorted, n, nq, qstart, qend);
}

__global__ void k_segments_align(const Align *__restrict__ s, uint32_t n, int32_t nq,
                                  uint32_t *__restrict__ qstart, uint32_t *__restrict__ qend)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (s[i].score <= 0) return;
    const int32_t q = s[i].q;
    if (i == 0 || s[i - 1].score <= 0 || s[i - 1].q != q) qstart[q] = i;
    if (i + 1 == n || s[i + 1].score <= 0 || s[i + 1].q != q) qend[q] = i + 1;
}

void launch_segments_align(const Align *sorted, uint32_t n, int32_t nq, uint32_t *qstart,
                           uint32_t *qend, hipStream_t st)
{
    if (n)
        k_segments_align<<<(n + kBlock - 1) / kBlock, kBlock, 0, st>>>(sorted, n, nq, qstart, qend);
}

__global__ void k_select_counts(const uint32_t *__restrict__ qstart,
                                const uint32_t *__restrict__ qend, int32_t nq, int32_t N,
                                uint32_t *__restrict__ nsel)
{
    const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    const uint32_t c = qend[q] - qstart[q];
    nsel[q] = (N > 0 && c > (uint32_t)N) ? (uint32_t)N : c;
}

// A replayed wave's per-query ranges and counts in one launch (no zero-fill, no
// per-record pass), thread ql for query ql of the nq_cap grid.  Runs are in query
// order, so a binary search finds each query's range; a query's selected boxes
// lead its own segment [seg_off[ql], seg_off[ql + 1]) (valid boxes sort first), so
// a binary search in the segment finds where they end.  counts[ql] is the range's
// length, capped at N when N > 0; queries past the wave, and flagged queries (their
// runs outgrew the LDS sort: the host runs them again), get empty ranges.
__global__ void k_cand_ranges(const Cand *__restrict__ c, int32_t nq_cap,
                              uint32_t *__restrict__ qstart, uint32_t *__restrict__ qend,
                              uint32_t *__restrict__ counts, uint32_t *__restrict__ off,
                              uint32_t *__restrict__ clear, const WaveCtl *__restrict__ ctl)
{
    const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q > nq_cap) return;
    const uint32_t n = ctl->nc;
    if (q == nq_cap) {
        off[q] = n;
        if (clear) *clear = 0u;
        return;
    }
    uint32_t a = n, b = n;  // queries past the wave: empty ranges at the end
    if (q < ctl->nqw && n > 0) {
        uint32_t lo = 0, hi = n;  // first run of query >= q
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (c[mid].q < q) lo = mid + 1;
            else hi = mid;
        }
        a = lo;
        hi = n;  // first run of query > q
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (c[mid].q <= q) lo = mid + 1;
            else hi = mid;
        }
        b = lo;
    }
    qstart[q] = a;
    qend[q] = b;
    counts[q] = b - a;
    off[q] = a;  // runs are in query order: a query's first run is its offset
}

__global__ void k_box_ranges(const Box *__restrict__ s, const uint32_t *__restrict__ seg_off,
                             int32_t nq_cap, int32_t N, uint32_t *__restrict__ qstart,
                             uint32_t *__restrict__ qend, uint32_t *__restrict__ counts,
                             const WaveCtl *__restrict__ ctl)
{
    const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq_cap) return;
    uint32_t a = 0, b = 0;
    if (q < ctl->nqw && !ctl->qflag[ctl->qa + q]) {
        a = seg_off[q];
        uint32_t lo = a, hi = seg_off[q + 1];  // first empty slot of the segment
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (s[mid].q >= 0) lo = mid + 1;
            else hi = mid;
        }
        b = lo;
    }
    qstart[q] = a;
    qend[q] = b;
    const uint32_t cnt = b - a;
    counts[q] = (N > 0 && cnt > (uint32_t)N) ? (uint32_t)N : cnt;
}

void launch_cand_ranges_ctl(const Cand *c, int32_t nq_cap, uint32_t *qstart, uint32_t *qend,
                            uint32_t *counts, uint32_t *off, uint32_t *clear, const WaveCtl *ctl,
                            hipStream_t st)
{
    k_cand_ranges<<<(nq_cap + kBlock) / kBlock, kBlock, 0, st>>>(c, nq_cap, qstart, qend, counts,
                                                                   off, clear, ctl);
}

// The same ranges, with the exclusive scan of the capped counts (sel_off[0..nq_cap],
// total last) in the same launch: one block of kRangeBlock threads, a query per
// thread (looping when there are more), so the segments' searches run side by side.
constexpr int kRangeBlock = 1024;

__global__ __launch_bounds__(kRangeBlock) void k_box_ranges_scan(
    const Box *__restrict__ s, const uint32_t *__restrict__ seg_off, int32_t nq_cap, int32_t N,
    uint32_t *__restrict__ qstart, uint32_t *__restrict__ qend, uint32_t *__restrict__ sel_off,
    uint32_t *__restrict__ sel_box, const WaveCtl *__restrict__ ctl)
{
    __shared__ uint32_t s_w[kRangeBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t carry = 0;
    for (int32_t q0 = 0; q0 < nq_cap; q0 += kRangeBlock) {
        const int32_t q = q0 + (int32_t)threadIdx.x;
        uint32_t a = 0, b = 0;
        if (q < nq_cap && q < ctl->nqw && !ctl->qflag[ctl->qa + q]) {
            a = seg_off[q];
            uint32_t lo = a, hi = seg_off[q + 1];  // first empty slot of the segment
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (s[mid].q >= 0) lo = mid + 1;
                else hi = mid;
            }
            b = lo;
        }
        const uint32_t cnt = (N > 0 && b - a > (uint32_t)N) ? (uint32_t)N : b - a;
        uint32_t x = cnt;  // block-wide exclusive scan of cnt
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) s_w[w] = x;
        __syncthreads();
        uint32_t before = 0, tot = 0;
#pragma unroll
        for (int i = 0; i < kRangeBlock / 64; ++i) {
            const uint32_t t = s_w[i];
            if (i < w) before += t;
            tot += t;
        }
        __syncthreads();
        const uint32_t ex = carry + before + x - cnt;
        if (q < nq_cap) {
            qstart[q] = a;
            qend[q] = b;
            sel_off[q] = ex;
            // the aligner's boxes, in selection order: the r-th is box a + r
            for (uint32_t r = 0; r < cnt; ++r) sel_box[ex + r] = a + r;
        }
        carry += tot;
    }
    if (threadIdx.x == 0) sel_off[nq_cap] = carry;
}

void launch_box_ranges_ctl(const Box *s, const uint32_t *seg_off, int32_t nq_cap, int32_t N,
                           uint32_t *qstart, uint32_t *qend, uint32_t *counts, const WaveCtl *ctl,
                           hipStream_t st)
{
    k_box_ranges<<<(nq_cap + kBlock - 1) / kBlock, kBlock, 0, st>>>(s, seg_off, nq_cap, N, qstart,
                                                                      qend, counts, ctl);
}

void launch_box_ranges_scan_ctl(const Box *s, const uint32_t *seg_off, int32_t nq_cap, int32_t N,
                                uint32_t *qstart, uint32_t *qend, uint32_t *sel_off,
                                uint32_t *sel_box, const WaveCtl *ctl, hipStream_t st)
{
    k_box_ranges_scan<<<1, kRangeBlock, 0, st>>>(s, seg_off, nq_cap, N, qstart, qend, sel_off,
                                                 sel_box, ctl);
}

void launch_select_counts(const uint32_t *qstart, const uint32_t *qend, int32_t nq,
                          int32_t max_hits, uint32_t *nsel, hipStream_t st)
{
    if (nq > 0)
        k_select_counts<<<(nq + kBlock - 1) / kBlock, kBlock, 0, st>>>(qstart, qend, nq, max_hits,
                                                                        nsel);
}

// ------------------------------------------------------------------ S9: banded Smith-Waterman
// One wave per selected box.  Cells are swept by anti-diagonal a = i + j.  On
// anti-diagonal a the band holds every other band diagonal t = j - i - c0 + W, all
// of one parity p; lane u owns t = p + 2u, so W + 1 lanes at most are busy.  The
// left neighbour (t - 1) and the upper neighbour (t + 1) were on anti-diagonal
// a - 1 in this lane or the adjacent one, and arrive by a one-lane DPP shift; the
// diagonal neighbour (same t) is this lane's own cell of a - 2.
//
// Each lane walks a staircase: after a step of parity 0 it moves one column
// right, after parity 1 one row down.  Every lane reads the query base and the
// two bank bases of its next pair one pair ahead, from the box's bases staged in
// LDS (or from global memory for boxes too long to stage).
// Starts and best cells are packed as i * 128 + t.
// Lanes without a source (lane 0, resp. lane 63) read 0; the kernel never uses them.
__device__ __forceinline__ int32_t from_lower_lane(int32_t v)  // lane u gets lane u - 1
{
    return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true);  // wave_shr:1
}
__device__ __forceinline__ int32_t from_upper_lane(int32_t v)  // lane u gets lane u + 1
{
    return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true);  // wave_shl:1
}

// In-band cells of an R x C box: band diagonals c = j - i in [clo, chi], each
// holding min(R, C - c) - max(0, -c) cells.  Lane-parallel over c, wave sum.
__device__ __forceinline__ unsigned long long band_cells(int32_t R, int32_t C, int32_t clo,
                                                         int32_t chi, int32_t lane)
{
    unsigned long long n = 0;
    for (int32_t c = clo + lane; c <= chi; c += 64) n += (uint32_t)(min(R, C - c) - max(0, -c));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) n += __shfl_xor(n, off, 64);
    return n;
}

// One cell of the affine recurrence with start tracking (see the oracle's O9):
// E/F open from the left/upper cell when the open term is >= the extend term;
// H > 0 takes its start from G (its diagonal predecessor's start, or itself if
// that H <= 0), else from E, else from F.  The start of a cell with H <= 0 is
// left as that rule gives it: no cell with H > 0 inherits it (the diagonal
// successor takes its own position, and a gap opened from H <= 0 is negative
// and stays so, as the penalties are >= 0), and only cells with H > 0 are
// reported.
struct CellOut {
    int32_t H, E, F, S, SE, SF;
};

__device__ __forceinline__ CellOut sw_cell(int32_t hl, int32_t el, int32_t sl, int32_t sel,
                                           int32_t hu, int32_t fu, int32_t su, int32_t sfu,
                                           int32_t hd, int32_t sd, bool same, int32_t here,
                                           int32_t match, int32_t mismatch, int32_t o1,
                                           int32_t ext)
{
    CellOut c;
    const int32_t eo = hl - o1, ee = el - ext;
    const bool eop = eo >= ee;
    c.E = eop ? eo : ee;
    c.SE = eop ? sl : sel;
    const int32_t fo = hu - o1, fe = fu - ext;
    const bool fop = fo >= fe;
    c.F = fop ? fo : fe;
    c.SF = fop ? su : sfu;
    const int32_t g = hd + (same ? match : -mismatch);
    c.H = max(max(g, 0), max(c.E, c.F));
    const int32_t sg = hd > 0 ? sd : here;
    c.S = (g == c.H) ? sg : ((c.E == c.H) ? c.SE : c.SF);
    return c;
}

// Cell with every value offset by kBswBias (the rest of the sweep after the border
// pairs, staged boxes): minus infinity is any value <= 0, so the zero that a DPP
// lane shift brings into lane 0 and lane 63 is one, and the shift can feed the
// subtraction or select that uses it.  The H floor is kBswBias; the score terms and
// gap costs come in as VGPRs.  The same rules as sw_cell otherwise.
constexpr int32_t kBswBias = 1 << 29;

__device__ __forceinline__ CellOut sw_cell_b(int32_t hl, int32_t el, int32_t sl, int32_t sel,
                                             int32_t hu, int32_t fu, int32_t su, int32_t sfu,
                                             int32_t hd, int32_t sd, bool same, int32_t here,
                                             int32_t vmatch, int32_t vmis, int32_t vo1,
                                             int32_t vext)
{
    CellOut c;
    const int32_t eo = hl - vo1, ee = el - vext;
    const bool eop = eo >= ee;
    c.E = eop ? eo : ee;
    c.SE = eop ? sl : sel;
    const int32_t fo = hu - vo1, fe = fu - vext;
    const bool fop = fo >= fe;
    c.F = fop ? fo : fe;
    c.SF = fop ? su : sfu;
    const int32_t g = hd + (same ? vmatch : vmis);
    c.H = max(max(g, kBswBias), max(c.E, c.F));
    const int32_t sg = hd > kBswBias ? sd : here;
    c.S = (g == c.H) ? sg : ((c.E == c.H) ? c.SE : c.SF);
    return c;
}

// A uniform value in a VGPR of its own (the compiler would otherwise rebuild it
// from its SGPR inside the loop, where two SGPR operands cannot meet in one select).
__device__ __forceinline__ int32_t in_vgpr(int32_t s)
{
    int32_t v;
    asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
    return v;
}

// The sweep over anti-diagonals [a0, a1] in pairs: X = the lane's cell of even
// parity (t = 2u) on a, Y = its cell of odd parity (t = 2u + 1) on a + 1, one
// column to the right.  X's left neighbour is the lower lane's previous Y, its
// upper neighbour this lane's previous Y, its diagonal this lane's previous X;
// Y's left neighbour is this lane's X, its upper the upper lane's X, its diagonal
// this lane's previous Y.  Lanes past the band (u > W) follow lane W's cells, so
// every base they read is in the box; no band cell reads their values.
// Staged bank bases come in pairs: sd2[x] holds base x and base min(x + 1, C - 1).
template <bool STAGED>
__device__ __forceinline__ void bsw_sweep(const uint8_t *__restrict__ sq,
                                          const uint16_t *__restrict__ sd2,
                                          const uint8_t *__restrict__ qp,
                                          const uint32_t *__restrict__ dbw, int64_t dbase,
                                          int32_t R, int32_t C, int32_t c0, int32_t W, int32_t a0,
                                          int32_t a1, int32_t match, int32_t mismatch, int32_t o1,
                                          int32_t ext, int32_t lane, int32_t &best,
                                          int32_t &bcell, int32_t &bstart)
{
    const int32_t tX = 2 * lane, tY = tX + 1;
    const bool laneX = tX <= 2 * W, laneY = tY <= 2 * W;
    const int32_t dXl = min(tX, 2 * W) - W + c0;  // the lane's X diagonal j - i
    int32_t i = (a0 - dXl) >> 1;
    int32_t j = a0 - i;
    int32_t hereX = i * 128 + tX;
    // the pair before the first, (i - 1, j - 1) and (i - 1, j), by the rule below: no
    // in-box cell of the band lies on its anti-diagonals, so it is border or -inf
    int32_t HX = (i < 1 || j < 1) ? 0 : kNegInf, EX = kNegInf, FX = kNegInf, SX = 0, SEX = 0,
            SFX = 0;
    int32_t HY = (i < 1 || j < 0) ? 0 : kNegInf, EY = kNegInf, FY = kNegInf, SY = 0, SEY = 0,
            SFY = 0;
    auto bases = [&](int32_t ii, int32_t jj, int32_t &qb, int32_t &dX, int32_t &dY) {
        const int32_t ic = min(max(ii, 0), R - 1);
        const int32_t jc = min(max(jj, 0), C - 1), jc1 = min(max(jj + 1, 0), C - 1);
        if (STAGED) {
            qb = sq[ic];
            dX = sd2[jc] & 0xff;
            dY = sd2[jc1] & 0xff;
        } else {
            qb = qp[ic];
            dX = db_base(dbw, dbase + jc);
            dY = db_base(dbw, dbase + jc1);
        }
    };
    int32_t nqb, ndX, ndY;  // bases of the next pair, read one pair ahead
    bases(i, j, nqb, ndX, ndY);
    // Every cell a lane computes follows one rule: a cell before the box (row or
    // column < 0) is the border (H = 0, E = F = -inf), a slot outside the band is
    // -inf, any other cell takes the recurrence.  In-box cells read only cells at or
    // before them, so this gives them exactly the box's borders and band; cells past
    // the box are never read and only kept out of the best cell.  The one neighbour
    // no lane holds, left of slot 0, is the border in column 0 and -inf elsewhere.
    // The first pairs hold cells before the box (row or column < 0); once every
    // band lane has reached row and column 0 (after `edge` pairs) no cell is, and
    // after one pair more slot 0's left neighbour is -inf for good: the rest of the
    // sweep drops the border tests.  There only the one lane whose Y slot lies past
    // the band (t = 2W + 1) is still forced to -inf, since its X reads it; other
    // slots past the band are read by no in-band cell.
    int32_t edge = (lane <= W) ? max(0, max(-i, -j)) : 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) edge = max(edge, __shfl_xor(edge, off, 64));
    edge = __builtin_amdgcn_readfirstlane(edge) + 1;
    auto pair = [&](auto edge_tag) {
        constexpr bool EDGE = decltype(edge_tag)::value;
        const int32_t qb = nqb, dX = ndX, dY = ndY;
        bases(i + 1, j + 1, nqb, ndX, ndY);
        const bool before_row = EDGE && i < 0;
        const bool rowin = (uint32_t)i < (uint32_t)R;
        {  // X = (i, j): left = the lower lane's previous Y, up = this lane's previous Y
            int32_t hl = from_lower_lane(HY), el = from_lower_lane(EY);
            const int32_t sl = from_lower_lane(SY), sel = from_lower_lane(SEY);
            if (lane == 0) {
                hl = j == 0 ? 0 : kNegInf;
                el = kNegInf;
            }
            const CellOut c = sw_cell(hl, el, sl, sel, HY, FY, SY, SFY, HX, SX, qb == dX, hereX,
                                      match, mismatch, o1, ext);
            if (EDGE) {
                const bool border = before_row || j < 0;
                HX = border ? 0 : (laneX ? c.H : kNegInf);
                EX = (border || !laneX) ? kNegInf : c.E;
                FX = (border || !laneX) ? kNegInf : c.F;
            } else {
                HX = c.H;
                EX = c.E;
                FX = c.F;
            }
            SX = c.S; SEX = c.SE; SFX = c.SF;
            if (laneX && rowin && (uint32_t)j < (uint32_t)C && c.H > best) {
                best = c.H;
                bcell = hereX;
                bstart = c.S;
            }
        }
        {  // Y = (i, j + 1): left = this lane's X, up = the upper lane's X
            const int32_t jy = j + 1;
            const int32_t hu = from_upper_lane(HX), fu = from_upper_lane(FX);
            const int32_t su = from_upper_lane(SX), sfu = from_upper_lane(SFX);
            const CellOut c = sw_cell(HX, EX, SX, SEX, hu, fu, su, sfu, HY, SY, qb == dY, hereX + 1,
                                      match, mismatch, o1, ext);
            if (EDGE) {
                const bool border = before_row || jy < 0;
                HY = border ? 0 : (laneY ? c.H : kNegInf);
                EY = (border || !laneY) ? kNegInf : c.E;
                FY = (border || !laneY) ? kNegInf : c.F;
            } else {
                HY = laneY ? c.H : kNegInf;
                EY = c.E;
                FY = laneY ? c.F : kNegInf;
            }
            SY = c.S; SEY = c.SE; SFY = c.SF;
            if (laneY && rowin && (uint32_t)jy < (uint32_t)C && c.H > best) {
                best = c.H;
                bcell = hereX + 1;
                bstart = c.S;
            }
        }
    };
    int32_t a = a0;
    for (const int32_t a_edge = a0 + 2 * edge; a <= a1 && a < a_edge; a += 2, ++i, ++j, hereX += 128)
        pair(std::true_type{});
    if constexpr (!STAGED) {
        for (; a <= a1; a += 2, ++i, ++j, hereX += 128) pair(std::false_type{});
    } else {
        // In the box's interior every band lane's row and column are >= 1, so the
        // bases need only the upper clamps, and X (resp. Y) lies in the box while a <
        // limX (limY): i < R and j < C (j + 1 < C) with i = (a - d) / 2, j = (a + d) / 2.
        const int32_t limX = laneX ? min(2 * R + dXl, 2 * C - dXl) : INT32_MIN;
        const int32_t limY = laneY ? min(2 * R + dXl, 2 * C - dXl - 2) : INT32_MIN;
        const int32_t vmatch = in_vgpr(match), vmis = in_vgpr(-mismatch), vo1 = in_vgpr(o1),
                      vext = in_vgpr(ext);
        HX += kBswBias; EX += kBswBias; FX += kBswBias;
        HY += kBswBias; EY += kBswBias; FY += kBswBias;
        int32_t bestb = best + kBswBias;
        // Bases two pairs ahead, in two sets that the pairs use in turn (even pairs
        // set 0, odd pairs set 1), so a read lands in the register its pair reads two
        // pairs later, with no copy waiting for it in between.
        // Bases two pairs ahead, in two sets that the pairs use in turn (even pairs
        // set 0, odd pairs set 1), so a read lands in the register its pair reads two
        // pairs later, with no copy waiting for it in between.
        auto fast_pair = [&](int32_t &nq, uint32_t &nd) {
            const int32_t qb = nq;
            const uint32_t dd = nd;
            nq = sq[min(i + 2, R - 1)];
            nd = sd2[min(j + 2, C - 1)];
            // keeps the reads here: without it the compiler moves them down to the pair
            // that uses them (nothing in the loop writes LDS) and waits for them there
            asm volatile("" ::: "memory");
            {  // X
                const CellOut c = sw_cell_b(from_lower_lane(HY), from_lower_lane(EY),
                                            from_lower_lane(SY), from_lower_lane(SEY), HY, FY, SY,
                                            SFY, HX, SX, qb == (int32_t)(dd & 0xffu), hereX,
                                            vmatch, vmis, vo1, vext);
                HX = c.H; EX = c.E; FX = c.F;
                SX = c.S; SEX = c.SE; SFX = c.SF;
                if (a < limX && c.H > bestb) {
                    bestb = c.H;
                    bcell = hereX;
                    bstart = c.S;
                }
            }
            {  // Y
                const CellOut c = sw_cell_b(HX, EX, SX, SEX, from_upper_lane(HX),
                                            from_upper_lane(FX), from_upper_lane(SX),
                                            from_upper_lane(SFX), HY, SY,
                                            qb == (int32_t)(dd >> 8), hereX + 1, vmatch, vmis,
                                            vo1, vext);
                HY = laneY ? c.H : 0;
                EY = c.E;
                FY = laneY ? c.F : 0;
                SY = c.S; SEY = c.SE; SFY = c.SF;
                if (a < limY && c.H > bestb) {
                    bestb = c.H;
                    bcell = hereX + 1;
                    bstart = c.S;
                }
            }
            a += 2;
            ++i;
            ++j;
            hereX += 128;
        };
        int32_t nq0 = sq[min(max(i, 0), R - 1)], nq1 = sq[min(max(i + 1, 0), R - 1)];
        uint32_t nd0 = sd2[min(max(j, 0), C - 1)], nd1 = sd2[min(max(j + 1, 0), C - 1)];
        // pairs in twos; an odd count ends with one pair past the box, whose cells
        // are out of it (a >= limX, limY) and read no base outside the staged ones
        while (a <= a1) {
            fast_pair(nq0, nd0);
            fast_pair(nq1, nd1);
        }
        best = bestb - kBswBias;
    }
}

// The b-th selected box and its wave query: named directly by sel_box, or the
// (b - sel_off[q])-th of query q's selection, q found by binary search.
__device__ __forceinline__ Box bsw_box(uint32_t b, const Box *__restrict__ sorted,
                                       const uint32_t *__restrict__ qstart,
                                       const uint32_t *__restrict__ sel_off, int32_t nq,
                                       const uint32_t *__restrict__ sel_box, int32_t &q)
{
    if (sel_box) {
        const Box bx = sorted[sel_box[b]];
        q = bx.q;
        return bx;
    }
    int32_t lo = 0, hi = nq - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (sel_off[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    q = lo;
    return sorted[qstart[q] + (b - sel_off[q])];
}

// Launch order of the aligner's boxes, longest first.  A box's sweep is one serial
// chain of about R + C anti-diagonals, so the longest boxes bound the kernel's
// time; listed first, they start at once and the short ones fill in around them.
// Boxes are classed by floor(log2(R + C)) (order within a class is arbitrary: each
// box writes its own output slot).  cnt[0..32) counts the classes, cnt[32..64)
// hands out slots within them; both start at zero.
constexpr int kOrderBlocks = 64;

__device__ __forceinline__ uint32_t bsw_class(const Box &bx)
{
    const uint32_t n = (uint32_t)max(bx.qe - bx.qs, 0) + (uint32_t)max(bx.de - bx.ds, 0);
    return n ? 31u - (uint32_t)__clz(n) : 0u;
}

__global__ __launch_bounds__(kBlock) void k_bsw_classes(
    const Box *__restrict__ sorted, const uint32_t *__restrict__ qstart,
    const uint32_t *__restrict__ sel_off, int32_t nq, uint32_t total,
    const uint32_t *__restrict__ sel_box, uint32_t *__restrict__ cnt,
    const WaveCtl *__restrict__ ctl)
{
    __shared__ uint32_t s_c[32];
    if (ctl) {
        nq = ctl->nqw;
        total = nq > 0 ? sel_off[nq] : 0;
    }
    if (threadIdx.x < 32) s_c[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t b = blockIdx.x * kBlock + threadIdx.x; b < total; b += gridDim.x * kBlock) {
        int32_t q;
        atomicAdd(&s_c[bsw_class(bsw_box(b, sorted, qstart, sel_off, nq, sel_box, q))], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 32 && s_c[threadIdx.x]) atomicAdd(&cnt[threadIdx.x], s_c[threadIdx.x]);
}

__global__ __launch_bounds__(kBlock) void k_bsw_order(
    const Box *__restrict__ sorted, const uint32_t *__restrict__ qstart,
    const uint32_t *__restrict__ sel_off, int32_t nq, uint32_t total,
    const uint32_t *__restrict__ sel_box, uint32_t *__restrict__ cnt,
    uint32_t *__restrict__ order, const WaveCtl *__restrict__ ctl)
{
    __shared__ uint32_t s_c[32], s_base[32];
    if (ctl) {
        nq = ctl->nqw;
        total = nq > 0 ? sel_off[nq] : 0;
    }
    const uint32_t stride = gridDim.x * kBlock;
    if (threadIdx.x < 32) s_c[threadIdx.x] = 0;
    __syncthreads();
    uint32_t cls[8], rank[8];  // a block's boxes: at most 8 per thread per sweep
    for (uint32_t b0 = blockIdx.x * kBlock; b0 < total; b0 += 8 * stride) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const uint32_t b = b0 + r * stride + threadIdx.x;
            cls[r] = 32;
            if (b < total) {
                int32_t q;
                cls[r] = bsw_class(bsw_box(b, sorted, qstart, sel_off, nq, sel_box, q));
                rank[r] = atomicAdd(&s_c[cls[r]], 1u);
            }
        }
        __syncthreads();
        if (threadIdx.x < 32) {  // the block's slots in each class, classes longest first
            uint32_t above = 0;
            for (uint32_t c = 31; c > threadIdx.x; --c) above += cnt[c];
            const uint32_t n = s_c[threadIdx.x];
            s_base[threadIdx.x] = n ? above + atomicAdd(&cnt[32 + threadIdx.x], n) : 0u;
            s_c[threadIdx.x] = 0;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 8; ++r)
            if (cls[r] < 32) order[s_base[cls[r]] + rank[r]] = b0 + r * stride + threadIdx.x;
        __syncthreads();
    }
}

// One wave (one block) per selected box; boxes whose bases fit kBswStage each
// for query and data bank are first staged in LDS.  Block i takes the order[i]-th
// box (the i-th without an order), then every gridDim.x-th after it.
__global__ __launch_bounds__(64) void k_bsw(
    const Box *__restrict__ sorted, const uint32_t *__restrict__ qstart,
    const uint32_t *__restrict__ sel_off, int32_t nq, uint32_t total,
    const uint8_t *__restrict__ qcode, const int64_t *__restrict__ qoff, int32_t qa,
    const uint32_t *__restrict__ dbw, const int64_t *__restrict__ seq_start, int32_t match,
    int32_t mismatch, int32_t o1, int32_t ext, int32_t W, Align *__restrict__ out,
    unsigned long long *__restrict__ cells_q, unsigned long long *__restrict__ cells_box,
    const uint32_t *__restrict__ sel_box, const uint32_t *__restrict__ order,
    const WaveCtl *__restrict__ ctl)
{
    __shared__ uint8_t s_q[kBswStage];
    __shared__ uint16_t s_d2[kBswStage];  // bank bases x and min(x + 1, C - 1)
    const int32_t lane = threadIdx.x;
    if (ctl) {
        nq = ctl->nqw;
        qa = ctl->qa;
        total = nq > 0 ? sel_off[nq] : 0;
    }
    for (uint32_t i = blockIdx.x; i < total; i += gridDim.x) {
    const uint32_t b = order ? order[i] : i;
    int32_t q;
    const Box bx = bsw_box(b, sorted, qstart, sel_off, nq, sel_box, q);
    const int32_t R = bx.qe - bx.qs, C = bx.de - bx.ds;
    const int32_t d0 = floor_half(bx.dmin + bx.dmax);
    const int32_t c0 = d0 - (bx.ds - bx.qs);  // cell (i, j) in band iff |j - i - c0| <= W
    const uint8_t *__restrict__ qp = qcode + qoff[qa + q] + bx.qs;
    const int64_t dbase = seq_start[bx.s] + bx.ds;
    const int32_t clo = max(c0 - W, -(R - 1)), chi = min(c0 + W, C - 1);
    int32_t best = 0, bcell = 0x7fffffff, bstart = 0;
    unsigned long long cells = 0;
    if (R > 0 && C > 0 && clo <= chi) {
        const int32_t a_lo = (clo <= 0 && chi >= 0) ? 0 : (clo > 0 ? clo : -chi);
        const int32_t cs = min(max(C - R, clo), chi);
        const int32_t a_hi = (cs <= C - R) ? 2 * (R - 1) + cs : 2 * (C - 1) - cs;
        // pairs start on an even-parity and end on an odd-parity anti-diagonal; the
        // extra anti-diagonals this may add hold no cell of the box
        const int32_t a0 = a_lo - ((a_lo - c0 + W) & 1);
        const int32_t a1 = a_hi + (((a_hi - c0 + W) & 1) ^ 1);
        cells = band_cells(R, C, clo, chi, lane);
        // a box's sweep is one serial chain of anti-diagonals, so the longest boxes
        // set the kernel's time: their waves take issue priority over short ones
        const int32_t span = a1 - a0;
        if (span > 1024) __builtin_amdgcn_s_setprio(3);
        else if (span > 512) __builtin_amdgcn_s_setprio(2);
        else if (span > 256) __builtin_amdgcn_s_setprio(1);
        if (R <= kBswStage && C <= kBswStage) {
            for (int32_t x = lane; x < R; x += 64) s_q[x] = qp[x];
            for (int32_t x = lane; x < C; x += 64)
                s_d2[x] = (uint16_t)(db_base(dbw, dbase + x) |
                                     (db_base(dbw, dbase + min(x + 1, C - 1)) << 8));
            __syncthreads();
            bsw_sweep<true>(s_q, s_d2, qp, dbw, dbase, R, C, c0, W, a0, a1, match, mismatch, o1,
                            ext, lane, best, bcell, bstart);
        } else {
            bsw_sweep<false>(s_q, s_d2, qp, dbw, dbase, R, C, c0, W, a0, a1, match, mismatch, o1,
                             ext, lane, best, bcell, bstart);
        }
    }
    __builtin_amdgcn_s_setprio(0);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int32_t ob = __shfl_xor(best, off, 64);
        const int32_t oc = __shfl_xor(bcell, off, 64);
        const int32_t os = __shfl_xor(bstart, off, 64);
        if (ob > best || (ob == best && oc < bcell)) {
            best = ob;
            bcell = oc;
            bstart = os;
        }
    }
    if (lane == 0) {
        Align r;
        r.q = q;
        r.seq_id = bx.s;
        r.score = best;
        if (best > 0) {
            const int32_t si = bstart >> 7, st = bstart & 127, bi = bcell >> 7, bt = bcell & 127;
            r.q_start = bx.qs + si;
            r.q_end = bx.qs + bi + 1;
            r.d_start = bx.ds + si + st - W + c0;
            r.d_end = bx.ds + bi + bt - W + c0 + 1;
        } else {
            r.q_start = r.q_end = r.d_start = r.d_end = -1;
        }
        r.box_q_start = bx.qs;
        r.box_q_end = bx.qe;
        r.box_d_start = bx.ds;
        r.box_d_end = bx.de;
        r.box_len = min(R, C);
        r.band_d0 = d0;
        out[b] = r;
        if (cells_q) atomicAdd(&cells_q[q], cells);
        if (cells_box) cells_box[b] = cells;
    }
    __syncthreads();  // the next box restages s_q and s_d2
    }
}

void launch_bsw(const Box *sorted, const uint32_t *qstart, const uint32_t *sel_off, int32_t nq,
                uint32_t nsel_total, const uint8_t *qcode, const int64_t *qoff, int32_t qa,
                const uint32_t *dbw, const int64_t *seq_start, int32_t match, int32_t mismatch,
                int32_t gap_open, int32_t gap_extend, int32_t band, Align *out,
                unsigned long long *cells_per_q, unsigned long long *cells_per_box, hipStream_t st,
                const WaveCtl *ctl, const uint32_t *sel_box, uint32_t *order_buf)
{
    // graph form: the wave's selection count is read on the device
    const uint32_t grid = ctl ? 8 * kStrideGrid : std::min<uint32_t>(nsel_total, kMaxGrid);
    if (grid == 0) return;
    uint32_t *order = nullptr;
    if (order_buf) {
        uint32_t *cnt = order_buf;
        order = order_buf + 64;
        launch_fill_u32(cnt, 64, 0u, st);
        k_bsw_classes<<<kOrderBlocks, kBlock, 0, st>>>(sorted, qstart, sel_off, nq, nsel_total,
                                                       sel_box, cnt, ctl);
        k_bsw_order<<<kOrderBlocks, kBlock, 0, st>>>(sorted, qstart, sel_off, nq, nsel_total,
                                                     sel_box, cnt, order, ctl);
    }
    k_bsw<<<grid, 64, 0, st>>>(sorted, qstart, sel_off, nq, nsel_total, qcode, qoff, qa, dbw,
                               seq_start, match, mismatch, gap_open + gap_extend, gap_extend, band,
                               out, cells_per_q, cells_per_box, sel_box, order, ctl);
}

// ------------------------------------------------------------------ traceback
// The path of each reported alignment (one wave per hit, grid-stride): the banded
// DP recomputed over the hit's rectangle [q_start, q_end) x [d_start, d_end) in the
// band |j - i - cc| <= W around the hit's band centre, row by row.  Row i's band
// slot t is column j = i + cc - W + t; a lane holds slots lane and lane + 64.  The
// horizontal gap of a row is a prefix maximum over its slots: E(t) = max over
// t' < t of H'(t') - o1 - ext (t - 1 - t'), with H' = max(0, G, F) (a gap opened
// after a gap never beats extending it when gap_open >= 0), then H = max(H', E).
// Each cell stores 4 bits: how H was reached (0 diagonal, 1 horizontal gap, 2
// vertical gap, 3 diagonal from a non-positive predecessor or H <= 0) and whether
// each gap was opened here (ties open).  Lane 0 then walks back from the end cell
// with the same priorities, rescoring as it goes, and writes the operations
// right-aligned in the hit's slot.  status[h] = 0 when the walk ends on the
// rectangle's first cell with the hit's score, 1 otherwise (not an alignment of
// this query, bank and scoring).
__global__ __launch_bounds__(64) void k_traceback(
    const int32_t *__restrict__ hits, int32_t n, const uint8_t *__restrict__ qascii, int64_t qlen,
    const uint32_t *__restrict__ dbw, const int64_t *__restrict__ seq_start, int32_t n_seqs,
    int32_t match, int32_t mismatch, int32_t o1, int32_t ext, int32_t W,
    const int64_t *__restrict__ dir_off, uint8_t *__restrict__ dirs,
    const int64_t *__restrict__ ops_off, char *__restrict__ ops, int32_t *__restrict__ ops_len,
    int32_t *__restrict__ status)
{
    constexpr int32_t NEG = kNegInf;
    constexpr int32_t LOW = -(1 << 30) - (1 << 28);  // below every score a scan can see
    const int32_t lane = threadIdx.x;
    __shared__ int32_t s_hend, s_bad;
    for (int32_t h = blockIdx.x; h < n; h += gridDim.x) {
        const int32_t *hr = hits + (size_t)h * kHitInts;
        const int32_t s = hr[0], score = hr[1], qs = hr[2], qe = hr[3], ds = hr[4], de = hr[5];
        const int32_t d0 = hr[11];
        const int32_t R = qe - qs, C = de - ds, cc = d0 - (ds - qs);
        if (lane == 0) {
            s_hend = NEG;
            s_bad = 0;
        }
        __syncthreads();
        // the host checked the query span and the sequence id; the bank span is
        // checked here, before any base is read
        const bool shape_ok = s >= 0 && s < n_seqs && qs >= 0 && R > 0 && (int64_t)qe <= qlen &&
                              ds >= 0 && C > 0 &&
                              (int64_t)de <= seq_start[s + 1] - seq_start[s] && score > 0 &&
                              (C - 1) - (R - 1) - cc <= W && (C - 1) - (R - 1) - cc >= -W;
        if (!shape_ok) {
            if (lane == 0) {
                ops_len[h] = 0;
                status[h] = 1;
            }
            __syncthreads();
            continue;
        }
        const uint8_t *qp = qascii + qs;
        const int64_t dbase = seq_start[s] + ds;
        uint8_t *drow = dirs + dir_off[h];
        int32_t hp1 = NEG, hp2 = NEG, fp1 = NEG, fp2 = NEG;  // previous row, slots lane, lane + 64
        int32_t bad = 0;
        for (int32_t i = 0; i < R; ++i) {
            const int32_t jb = i + cc - W;  // column of slot 0
            const int32_t qb = base_code(qp[i]);
            bad |= qb < 0;
            // up neighbours: slot t + 1 of the previous row
            const int32_t up1h = __shfl_down(hp1, 1, 64), up1f = __shfl_down(fp1, 1, 64);
            const int32_t up2h = __shfl_down(hp2, 1, 64), up2f = __shfl_down(fp2, 1, 64);
            const int32_t wrap_h = __shfl(hp2, 0, 64), wrap_f = __shfl(fp2, 0, 64);
            int32_t hv[2], ev[2], fv[2], gv[2], dg[2], fo[2], tt[2], jj[2];
            bool ok[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                const int32_t t = lane + 64 * x;
                const int32_t j = jb + t;
                tt[x] = t;
                jj[x] = j;
                ok[x] = t <= 2 * W && j >= 0 && j < C;
                const int32_t hprev = x ? hp2 : hp1;
                int32_t uh = x ? (lane == 63 ? NEG : up2h) : (lane == 63 ? wrap_h : up1h);
                int32_t uf = x ? (lane == 63 ? NEG : up2f) : (lane == 63 ? wrap_f : up1f);
                if (i == 0) {
                    uh = 0;
                    uf = NEG;
                }
                const int32_t dh = (i == 0 || j == 0) ? 0 : hprev;
                int32_t g = NEG, f = NEG, hpr = NEG;
                fo[x] = 0;
                if (ok[x]) {
                    const int32_t db = db_base(dbw, dbase + j);
                    g = dh + (qb == db ? match : -mismatch);
                    f = max(uh - o1, uf - ext);
                    fo[x] = (uh - o1 >= uf - ext) ? 1 : 0;
                    hpr = max(max(0, g), f);
                }
                gv[x] = g;
                dg[x] = dh;
                fv[x] = f;
                hv[x] = hpr;
            }
            // horizontal gaps: exclusive prefix maximum of H'(t) + ext t over the slots
            int32_t a1 = ok[0] ? hv[0] + ext * tt[0] : LOW;
            int32_t a2 = ok[1] ? hv[1] + ext * tt[1] : LOW;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int32_t b1 = __shfl_up(a1, off, 64), b2 = __shfl_up(a2, off, 64);
                if (lane >= off) {
                    a1 = max(a1, b1);
                    a2 = max(a2, b2);
                }
            }
            const int32_t tot1 = __shfl(a1, 63, 64);
            int32_t pm1 = __shfl_up(a1, 1, 64), pm2 = __shfl_up(a2, 1, 64);
            if (lane == 0) {
                pm1 = LOW;
                pm2 = LOW;
            }
            pm2 = max(pm2, tot1);
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                const int32_t pm = x ? pm2 : pm1;
                ev[x] = (ok[x] && pm > LOW) ? max(pm - o1 - ext * (tt[x] - 1), NEG - ext) : NEG;
                if (ok[x]) hv[x] = max(hv[x], ev[x]);
            }
            // left neighbours: slot t - 1 of this row
            int32_t l1h = __shfl_up(hv[0], 1, 64), l1e = __shfl_up(ev[0], 1, 64);
            int32_t l2h = __shfl_up(hv[1], 1, 64), l2e = __shfl_up(ev[1], 1, 64);
            const int32_t w2h = __shfl(hv[0], 63, 64), w2e = __shfl(ev[0], 63, 64);
            if (lane == 0) {
                l1h = NEG;
                l1e = NEG;
                l2h = w2h;
                l2e = w2e;
            }
            uint8_t byte = 0;
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                int32_t lh = x ? l2h : l1h, le = x ? l2e : l1e;
                if (jj[x] == 0) {
                    lh = 0;
                    le = NEG;
                }
                const int32_t eo = (lh - o1 >= le - ext) ? 1 : 0;
                int32_t src = 3;
                if (ok[x] && hv[x] > 0) {
                    if (gv[x] == hv[x]) src = dg[x] > 0 ? 0 : 3;
                    else if (ev[x] == hv[x]) src = 1;
                    else src = 2;
                }
                const uint8_t nib = (uint8_t)(src | (eo << 2) | (fo[x] << 3));
                byte |= (uint8_t)(nib << (4 * x));
                if (ok[x] && i == R - 1 && jj[x] == C - 1) s_hend = hv[x];
            }
            drow[(size_t)i * 64 + lane] = byte;
            hp1 = ok[0] ? hv[0] : NEG;
            hp2 = ok[1] ? hv[1] : NEG;
            fp1 = ok[0] ? fv[0] : NEG;
            fp2 = ok[1] ? fv[1] : NEG;
        }
        if (bad) s_bad = 1;
        __threadfence_block();
        __syncthreads();
        if (lane == 0) {
            bool good = s_hend == score && !s_bad;
            const volatile uint8_t *vd = drow;
            char *o = ops + ops_off[h];
            const int64_t cap = (int64_t)R + C;
            int32_t i = R - 1, j = C - 1, state = 0;
            int64_t k = 0;
            int64_t sum = 0;
            while (good) {
                const int32_t t = j - (i + cc - W);
                if (i < 0 || j < 0 || k >= cap || t < 0 || t > 2 * W) {
                    good = false;
                    break;
                }
                const uint8_t nib = (uint8_t)(vd[(size_t)i * 64 + (t & 63)] >> (4 * (t >> 6))) & 15u;
                if (state == 0) {
                    const int32_t src = nib & 3;
                    if (src == 0 || src == 3) {
                        const bool eq = base_code(qp[i]) == db_base(dbw, dbase + j);
                        o[cap - 1 - k++] = eq ? '=' : 'X';
                        sum += eq ? match : -mismatch;
                        if (src == 3) {
                            good = i == 0 && j == 0;
                            break;
                        }
                        --i;
                        --j;
                    } else {
                        state = src;
                    }
                } else if (state == 1) {
                    o[cap - 1 - k++] = 'D';
                    const bool opened = (nib >> 2) & 1u;
                    sum -= opened ? o1 : ext;
                    state = opened ? 0 : 1;
                    --j;
                } else {
                    o[cap - 1 - k++] = 'I';
                    const bool opened = (nib >> 3) & 1u;
                    sum -= opened ? o1 : ext;
                    state = opened ? 0 : 2;
                    --i;
                }
            }
            good = good && sum == score;
            ops_len[h] = good ? (int32_t)k : 0;
            status[h] = good ? 0 : 1;
        }
        __syncthreads();
    }
}

void launch_traceback(const int32_t *hits, int32_t n, const uint8_t *qascii, int64_t qlen,
                      const uint32_t *dbw, const int64_t *seq_start, int32_t n_seqs, int32_t match,
                      int32_t mismatch, int32_t gap_open, int32_t gap_extend, int32_t band,
                      const int64_t *dir_off, uint8_t *dirs, const int64_t *ops_off, char *ops,
                      int32_t *ops_len, int32_t *status, hipStream_t st)
{
    if (n <= 0) return;
    const uint32_t grid = std::min<uint32_t>((uint32_t)n, kMaxGrid);
    k_traceback<<<grid, 64, 0, st>>>(hits, n, qascii, qlen, dbw, seq_start, n_seqs, match,
                                     mismatch, gap_open + gap_extend, gap_extend, band, dir_off,
                                     dirs, ops_off, ops, ops_len, status);
}

// Offsets of each hit's direction rows (64 bytes per query row of its rectangle),
// from the hits themselves, for callers that keep no host copy of them: one
// thread walks the hits in order.
__global__ void k_dir_offsets(const int32_t *__restrict__ hits, int32_t n,
                              int64_t *__restrict__ dir_off)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int64_t acc = 0;
    for (int32_t h = 0; h < n; ++h) {
        dir_off[h] = acc;
        const int32_t *hr = hits + (size_t)h * kHitInts;
        acc += 64 * (int64_t)max(hr[3] - hr[2], 0);
    }
    dir_off[n] = acc;
}

// ops_len[h] = -1 where the walk failed (status 1), so one array carries both.
__global__ void k_fold_status(int32_t *__restrict__ ops_len, const int32_t *__restrict__ status,
                              int32_t n)
{
    const int32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h < n && status[h] != 0) ops_len[h] = -1;
}

void launch_dir_offsets(const int32_t *hits, int32_t n, int64_t *dir_off, hipStream_t st)
{
    k_dir_offsets<<<1, 64, 0, st>>>(hits, n, dir_off);
}

void launch_fold_status(int32_t *ops_len, const int32_t *status, int32_t n, hipStream_t st)
{
    if (n <= 0) return;
    k_fold_status<<<(uint32_t)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(ops_len, status, n);
}

// ------------------------------------------------------------------ results to device memory
// One block per query: its first min(cap, n) ordered alignments become gg_hit
// records at out[q * cap], and its count goes to n_out[q].
__global__ void k_write_out(const Align *__restrict__ sorted, const uint32_t *__restrict__ rstart,
                            const uint32_t *__restrict__ rend, int32_t qa, int32_t cap,
                            int32_t *__restrict__ out, int32_t *__restrict__ n_out)
{
    const int32_t ql = blockIdx.x;
    const uint32_t a = rstart[ql], n = rend[ql] - a;
    if (threadIdx.x == 0) n_out[qa + ql] = (int32_t)n;
    const uint32_t m = min(n, (uint32_t)cap);
    int32_t *dst = out + ((size_t)(qa + ql) * (size_t)cap) * kHitInts;
    const int32_t *src = reinterpret_cast<const int32_t *>(sorted + a);
    for (uint32_t e = threadIdx.x; e < m * kHitInts; e += blockDim.x)
        dst[e] = src[(e / kHitInts) * kAlignInts + 1 + e % kHitInts];
}

void launch_write_out(const Align *sorted, const uint32_t *rstart, const uint32_t *rend,
                      int32_t nq, int32_t qa, int32_t cap, int32_t *out, int32_t *n_out,
                      hipStream_t st)
{
    if (nq > 0) k_write_out<<<nq, kBlock, 0, st>>>(sorted, rstart, rend, qa, cap, out, n_out);
}

}  // namespace gg
