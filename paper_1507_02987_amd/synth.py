"""Seeded synthetic workloads shaped like the paper's experiments (Section 5).

The paper searched a human-genome data bank plus RefSeq banks (about 4.25 Gb) with
query sets built from one data-bank sequence and ten mutated copies, from 80 bp to
1 Mbp.  Those files are not available, so this module draws stand-ins with the
same shape: sizes, length mixes, composition, repeats and planted homologs.

This module only draws random bytes.  It holds none of the search method's
arithmetic: no base coding, no k-mers, no scoring.  The oracle tests and the GPU
path both consume what it returns, so it imports nothing from either of them.

Everything is a pure function of ``ROOT_SEED`` and the workload's stream id, through
``numpy.random.Generator(PCG64(SeedSequence(ROOT_SEED)))`` children.
"""
from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

ROOT_SEED = 150702987
ASCII = np.frombuffer(b"ACGT", dtype=np.uint8)
# For a letter index 0..3 (A, C, G, T), the three other letters.
_OTHERS = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]], dtype=np.uint8)
_LUT = np.full(256, 255, dtype=np.uint8)
for _i, _c in enumerate(b"ACGT"):
    _LUT[_c] = _i


@dataclass
class Database:
    """Concatenated ASCII data-bank sequences: sequence s is seqs[off[s]:off[s+1]]."""

    seqs: np.ndarray  # uint8 ASCII
    off: np.ndarray  # int64, n_seqs + 1
    name: str = ""

    @property
    def n_seqs(self) -> int:
        return int(self.off.shape[0] - 1)

    @property
    def total_bp(self) -> int:
        return int(self.off[-1])

    def seq(self, s: int) -> np.ndarray:
        return self.seqs[self.off[s]:self.off[s + 1]]


@dataclass
class QuerySet:
    """Concatenated ASCII queries plus where each planted homolog came from."""

    buf: np.ndarray  # uint8 ASCII
    off: np.ndarray  # int64, n_queries + 1
    kind: np.ndarray  # int8: 1 planted homolog, 0 uniform random
    src_seq: np.ndarray  # int64, -1 for random queries
    src_start: np.ndarray  # int64
    src_end: np.ndarray  # int64
    identity: np.ndarray = field(default_factory=lambda: np.zeros(0))

    @property
    def n(self) -> int:
        return int(self.off.shape[0] - 1)

    def query(self, i: int) -> np.ndarray:
        return self.buf[self.off[i]:self.off[i + 1]]

    def lengths(self) -> np.ndarray:
        return np.diff(self.off)

    def subset(self, idx) -> "QuerySet":
        idx = np.asarray(idx, dtype=np.int64)
        parts = [self.query(int(i)) for i in idx]
        lens = np.array([len(p) for p in parts], dtype=np.int64)
        off = np.zeros(len(parts) + 1, dtype=np.int64)
        np.cumsum(lens, out=off[1:])
        buf = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
        ident = self.identity[idx] if self.identity.size else self.identity
        return QuerySet(buf, off, self.kind[idx], self.src_seq[idx], self.src_start[idx],
                        self.src_end[idx], ident)


# --------------------------------------------------------------------------- streams

def _streams(cfg_id: int):
    """Independent generators for (data bank, queries, arrivals) of one workload.

    The short-query and served sets search the large bank, so they take its stream.
    """
    root = np.random.SeedSequence(ROOT_SEED)
    per_cfg = root.spawn(5)
    db_ss, q_ss, arr_ss = per_cfg[cfg_id].spawn(3)
    if cfg_id in (3, 4):
        db_ss = per_cfg[2].spawn(3)[0]
    mk = lambda ss: np.random.Generator(np.random.PCG64(ss))
    return mk(db_ss), mk(q_ss), mk(arr_ss)


# --------------------------------------------------------------------------- helpers

def _uniform_bases(rng, n: int) -> np.ndarray:
    return ASCII[rng.integers(0, 4, size=n, dtype=np.uint8)]


def _gc_bases(rng, lengths: np.ndarray, gc: np.ndarray, chunk: int = 1 << 25) -> np.ndarray:
    """Bases with per-sequence GC fraction: P(G)=P(C)=gc/2, P(A)=P(T)=(1-gc)/2.

    One float32 uniform per base, drawn in order; base = number of the sequence's
    three thresholds (1-gc)/2, (1-gc)/2 + gc/2, (1-gc)/2 + gc that it reaches.
    The draws are sequential, the threshold tests run on a thread pool.
    """
    total = int(lengths.sum())
    out = np.empty(total, dtype=np.uint8)
    off = _offsets(lengths)
    g = gc.astype(np.float32)
    a = (1.0 - g) * 0.5
    thr = (a, a + g * 0.5, a + g)

    def fill(lo, u):
        hi = lo + len(u)
        # sequences overlapping [lo, hi) and how many of their bases fall inside
        s0 = int(np.searchsorted(off, lo, side="right")) - 1
        s1 = int(np.searchsorted(off, hi, side="left"))
        part = np.minimum(off[s0 + 1:s1 + 1], hi) - np.maximum(off[s0:s1], lo)
        idx = np.zeros(len(u), dtype=np.uint8)
        for t in thr:
            idx += u >= np.repeat(t[s0:s1], part)
        out[lo:hi] = ASCII[idx]

    with ThreadPoolExecutor(max_workers=8) as pool:
        pending = []
        for lo in range(0, total, chunk):
            pending.append(pool.submit(fill, lo, rng.random(min(total, lo + chunk) - lo,
                                                            dtype=np.float32)))
            if len(pending) >= 16:
                pending.pop(0).result()
        for f in pending:
            f.result()
    return out


def _offsets(lengths: np.ndarray) -> np.ndarray:
    off = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(lengths, out=off[1:])
    return off


def mutate(src: np.ndarray, sub_rate: float, indel_rate: float, rng) -> np.ndarray:
    """Copy ``src`` left to right with point substitutions and short indels.

    At each source position: with probability ``indel_rate`` an indel (insertion or
    deletion with equal odds, length uniform in 1..3, inserted letters uniform);
    otherwise with probability ``sub_rate`` a substitution to one of the three other
    letters; otherwise a plain copy.  An insertion emits its letters and then the
    source letter; a deletion skips that many source letters.
    """
    n = len(src)
    u_indel = rng.random(n)
    u_sub = rng.random(n)
    pick = rng.integers(0, 3, size=n, dtype=np.uint8)
    is_ins = rng.random(n) < 0.5
    ilen = rng.integers(1, 4, size=n)
    is_indel = u_indel < indel_rate
    is_sub = (~is_indel) & (u_sub < sub_rate)
    sub = src.copy()
    if is_sub.any():
        letters = _LUT[src[is_sub]]
        sub[is_sub] = ASCII[_OTHERS[letters, pick[is_sub]]]
    parts = []
    p = 0
    for ip in np.flatnonzero(is_indel):
        ip = int(ip)
        if ip < p:
            continue
        parts.append(sub[p:ip])
        ln = int(ilen[ip])
        if is_ins[ip]:
            parts.append(_uniform_bases(rng, ln))
            parts.append(src[ip:ip + 1])
            p = ip + 1
        else:
            p = ip + ln
    parts.append(sub[p:])
    return np.concatenate(parts)


def _pick_source(rng, db: Database, L: int, lens: np.ndarray, cum_cache: dict):
    """A data-bank sequence with probability proportional to length among those of
    length >= L, and a uniform start inside it."""
    key = L
    if key not in cum_cache:
        ok = np.flatnonzero(lens >= L)
        w = lens[ok].astype(np.float64)
        cum_cache[key] = (ok, np.cumsum(w) / w.sum())
    ok, cum = cum_cache[key]
    if len(ok) == 0:
        return -1, 0
    s = int(ok[min(int(np.searchsorted(cum, rng.random(), side="right")), len(ok) - 1)])
    start = int(rng.integers(0, int(lens[s]) - L + 1))
    return s, start


def _log_uniform_int(rng, lo: int, hi: int, n: int) -> np.ndarray:
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=n))).astype(np.int64)


def _queries(rng, db: Database, lengths: np.ndarray, homolog: np.ndarray, ident: np.ndarray,
             indel_rate: float) -> QuerySet:
    lens = np.diff(db.off)
    cache: dict = {}
    parts, src_seq, src_start, src_end = [], [], [], []
    for i, L in enumerate(lengths):
        L = int(L)
        if homolog[i]:
            s, st = _pick_source(rng, db, L, lens, cache)
            if s < 0:
                homolog[i] = 0
        if homolog[i]:
            region = db.seqs[db.off[s] + st: db.off[s] + st + L]
            parts.append(mutate(region, 1.0 - float(ident[i]), indel_rate, rng))
            src_seq.append(s)
            src_start.append(st)
            src_end.append(st + L)
        else:
            parts.append(_uniform_bases(rng, L))
            src_seq.append(-1)
            src_start.append(-1)
            src_end.append(-1)
    qlens = np.array([len(p) for p in parts], dtype=np.int64)
    return QuerySet(np.concatenate(parts), _offsets(qlens), homolog.astype(np.int8),
                    np.array(src_seq, np.int64), np.array(src_start, np.int64),
                    np.array(src_end, np.int64), np.where(homolog, ident, 0.0))


# --------------------------------------------------------------------------- small (stream 0)

def small_db(n_seqs: int = 2000) -> Database:
    """2,000 sequences, lengths uniform 200..2,000, i.i.d. uniform ACGT (about 2.2 Mbp)."""
    rng, _, _ = _streams(0)
    lengths = rng.integers(200, 2001, size=n_seqs).astype(np.int64)
    return Database(_uniform_bases(rng, int(lengths.sum())), _offsets(lengths), "small")


def small_queries(db: Database, n_homolog: int = 10, n_random: int = 10, L: int = 500) -> QuerySet:
    """Ten 500 bp data-bank regions with 5% substitutions and 1% indels, then ten
    uniform random 500 bp queries."""
    _, rng, _ = _streams(0)
    n = n_homolog + n_random
    homolog = np.array([1] * n_homolog + [0] * n_random, dtype=np.int8)
    ident = np.full(n, 0.95)
    return _queries(rng, db, np.full(n, L, np.int64), homolog, ident, 0.01)


# --------------------------------------------------------------------------- mid-size (stream 1)

def mid_db(n_seqs: int = 200_000) -> Database:
    """Lengths clip(round(LogNormal(ln 1000, 0.8)), 100, 50,000); per-sequence GC
    fraction uniform in 0.35..0.65 (about 275 Mbp at 200,000 sequences)."""
    rng, _, _ = _streams(1)
    lengths = np.clip(np.rint(rng.lognormal(math.log(1000.0), 0.8, size=n_seqs)), 100, 50_000)
    lengths = lengths.astype(np.int64)
    gc = rng.uniform(0.35, 0.65, size=n_seqs)
    return Database(_gc_bases(rng, lengths, gc), _offsets(lengths), "mid")


def mid_queries(db: Database, n: int = 1000, lmin: int = 80, lmax: int = 10_000) -> QuerySet:
    """Lengths log-uniform 80..10,000; half planted homologs at identity uniform in
    0.70..0.99 plus 1% indels, half uniform random, in a seeded shuffled order."""
    _, rng, _ = _streams(1)
    lengths = _log_uniform_int(rng, lmin, lmax, n)
    homolog = np.zeros(n, dtype=np.int8)
    homolog[: n // 2] = 1
    rng.shuffle(homolog)
    ident = rng.uniform(0.70, 0.99, size=n)
    return _queries(rng, db, lengths, homolog, ident, 0.01)


# --------------------------------------------------------------------------- large bank (stream 2)

def large_db(n_seqs: int = 500_000, chunk_seqs: int = 25_000) -> Database:
    """Lengths clip(round(LogNormal(ln 4000, 0.9)), 100, 200,000) (about 3 Gbp at
    500,000 sequences), per-sequence GC as the mid-size bank, then two repeat overlays:

    * interspersed repeats: 50 random 300 bp family consensi; each sequence of
      length n gets floor(0.05 n / 300) copies plus one more with probability of the
      fractional part, each copy with 10% substitutions, at uniform offsets;
    * tandem repeats: period uniform 1..6, random unit, length uniform 20..300, at
      uniform offsets, drawn until their summed length reaches 10% of the sequence.
    """
    rng, _, _ = _streams(2)
    lengths = np.clip(np.rint(rng.lognormal(math.log(4000.0), 0.9, size=n_seqs)), 100, 200_000)
    lengths = lengths.astype(np.int64)
    gc = rng.uniform(0.35, 0.65, size=n_seqs)
    seqs = _gc_bases(rng, lengths, gc)
    off = _offsets(lengths)
    families = _LUT[_uniform_bases(rng, 50 * 300)].reshape(50, 300)
    for lo in range(0, n_seqs, chunk_seqs):
        hi = min(n_seqs, lo + chunk_seqs)
        ln = lengths[lo:hi]
        # interspersed family copies
        x = 0.05 * ln / 300.0
        ncopy = np.floor(x).astype(np.int64) + (rng.random(hi - lo) < (x - np.floor(x)))
        ncopy[ln < 300] = 0
        tot = int(ncopy.sum())
        if tot:
            owner = np.repeat(np.arange(lo, hi), ncopy)
            fam = rng.integers(0, 50, size=tot)
            start = (rng.random(tot) * (lengths[owner] - 300 + 1)).astype(np.int64)
            body = families[fam].copy()
            subm = rng.random(body.shape) < 0.10
            pick = rng.integers(0, 3, size=body.shape, dtype=np.uint8)
            body[subm] = _OTHERS[body[subm], pick[subm]]
            pos = (off[owner] + start)[:, None] + np.arange(300)[None, :]
            seqs[pos.ravel()] = ASCII[body.ravel()]
        # tandem repeats: a pool per sequence, keep the prefix reaching 10% of it
        need = 0.10 * ln
        pool = np.ceil(need / 160.0 * 1.6).astype(np.int64) + 2
        owner = np.repeat(np.arange(lo, hi), pool)
        rlen = np.minimum(rng.integers(20, 301, size=len(owner)), lengths[owner])
        period = rng.integers(1, 7, size=len(owner))
        unit = rng.integers(0, 4, size=(len(owner), 6), dtype=np.uint8)
        first = np.zeros(hi - lo, dtype=np.int64)
        np.cumsum(pool[:-1], out=first[1:])
        csum = np.cumsum(rlen)
        base_before = csum[first] - rlen[first]
        prefix = csum - np.repeat(base_before, pool)  # inclusive sum within the owner
        keep = (prefix - rlen) < np.repeat(need, pool)
        owner, rlen, period, unit = owner[keep], rlen[keep], period[keep], unit[keep]
        start = (rng.random(len(owner)) * (lengths[owner] - rlen + 1)).astype(np.int64)
        rid = np.repeat(np.arange(len(owner)), rlen)
        rfirst = np.zeros(len(owner), dtype=np.int64)
        np.cumsum(rlen[:-1], out=rfirst[1:])
        t = np.arange(len(rid)) - rfirst[rid]
        letters = unit[rid, t % period[rid]]
        seqs[off[owner][rid] + start[rid] + t] = ASCII[letters]
    return Database(seqs, off, "large")


def large_queries(db: Database, n: int = 2000) -> QuerySet:
    """Lengths log-uniform 500..5,000; half planted homologs at identity uniform in
    0.75..0.99 plus 1% indels, half uniform random."""
    _, rng, _ = _streams(2)
    lengths = _log_uniform_int(rng, 500, 5000, n)
    homolog = np.zeros(n, dtype=np.int8)
    homolog[: n // 2] = 1
    rng.shuffle(homolog)
    ident = rng.uniform(0.75, 0.99, size=n)
    return _queries(rng, db, lengths, homolog, ident, 0.01)


# --------------------------------------------------------------------------- large bank, short queries (stream 3)

def large_short_queries(db: Database, n: int = 100_000) -> QuerySet:
    """Lengths uniform 100..250; 80% data-bank regions with 1..3% substitutions and
    no indels, 20% uniform random."""
    _, rng, _ = _streams(3)
    lengths = rng.integers(100, 251, size=n).astype(np.int64)
    homolog = (rng.random(n) < 0.8).astype(np.int8)
    ident = 1.0 - rng.uniform(0.01, 0.03, size=n)
    return _queries(rng, db, lengths, homolog, ident, 0.0)


# --------------------------------------------------------------------------- large bank, served (stream 4)

def large_served_queries(db: Database, n: int = 2000) -> QuerySet:
    """Lengths log-uniform 50..20,000; 60% planted homologs at identity uniform in
    0.75..0.99 plus 1% indels, 40% uniform random."""
    _, rng, _ = _streams(4)
    lengths = _log_uniform_int(rng, 50, 20_000, n)
    homolog = (rng.random(n) < 0.6).astype(np.int8)
    ident = rng.uniform(0.75, 0.99, size=n)
    return _queries(rng, db, lengths, homolog, ident, 0.01)


def served_arrivals(rate_per_s: float, n: int = 2000) -> np.ndarray:
    """Open-loop Poisson arrival times (seconds from 0) at the given rate; each rate
    has its own child of the served set's arrivals stream."""
    ss = np.random.SeedSequence(ROOT_SEED).spawn(5)[4].spawn(3)[2]
    child = np.random.SeedSequence(ss.entropy, spawn_key=ss.spawn_key + (int(rate_per_s),))
    rng = np.random.Generator(np.random.PCG64(child))
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))


# --------------------------------------------------------------------------- small DBs

def random_db(seed: int, n_seqs: int, lmin: int, lmax: int) -> Database:
    """A tiny i.i.d. uniform data bank for unit tests."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([ROOT_SEED, 7, seed])))
    lengths = rng.integers(lmin, lmax + 1, size=n_seqs).astype(np.int64)
    return Database(_uniform_bases(rng, int(lengths.sum())), _offsets(lengths), f"random{seed}")


def repeat_db(seed: int, n_seqs: int, lmin: int, lmax: int, frac_repeat: float = 0.3) -> Database:
    """A tiny uniform data bank where about frac_repeat of the sequences carry one
    tandem repeat (unit of 1-4 bases, 30-400 bases long) at a uniform offset, so a
    few posting lists grow long, as low-complexity regions make them."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([ROOT_SEED, 9, seed])))
    lengths = rng.integers(lmin, lmax + 1, size=n_seqs).astype(np.int64)
    seqs = _uniform_bases(rng, int(lengths.sum()))
    off = _offsets(lengths)
    for s in range(n_seqs):
        n = int(lengths[s])
        if n < 30 or rng.random() >= frac_repeat:
            continue
        unit = _uniform_bases(rng, int(rng.integers(1, 5)))
        rl = int(rng.integers(30, min(400, n) + 1))
        at = int(off[s]) + int(rng.integers(0, n - rl + 1))
        seqs[at:at + rl] = np.resize(unit, rl)
    return Database(seqs, off, f"repeat{seed}")


def random_queries(seed: int, db: Database, n: int, lmin: int, lmax: int, frac_homolog: float,
                   ident_lo: float, ident_hi: float, indel_rate: float) -> QuerySet:
    """Tiny mixed query sets for unit and parity tests."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([ROOT_SEED, 8, seed])))
    lengths = rng.integers(lmin, lmax + 1, size=n).astype(np.int64)
    homolog = (rng.random(n) < frac_homolog).astype(np.int8)
    ident = rng.uniform(ident_lo, ident_hi, size=n)
    return _queries(rng, db, lengths, homolog, ident, indel_rate)


TOP_N = {0: 20, 1: 50, 2: 100, 3: 20, 4: 50}
