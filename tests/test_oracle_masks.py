"""Pins of the oracle's spaced-seed masks (Section 2.1): windows of the mask's
length, coded on the bases under its 1s.

* the paper's mask 111010010100110111 on hand-worked windows (tests/golden/masks.json)
  against the plain k-base coding of the kept bases;
* the index size the paper states for an 18-base mask on 4 billion bases;
* an all-ones mask of length k equals the unmasked index and search;
* every hit equals a brute-force comparison of masked strings on tiny banks;
* an exact copy of a bank region is found whole with a mask.
"""
import json
import os

import numpy as np
import pytest

from paper_1507_02987_amd import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "masks.json")))


def test_paper_mask_worked_windows(ggo):
    m = GOLD["paper_mask"]
    assert len(m) == GOLD["span"] and m.count("1") == GOLD["weight"]
    for w in GOLD["worked"]:
        assert [t for t, ch in enumerate(m) if ch == "1"] == w["kept_positions"]
        got = ggo.masked_code(ggo.encode(w["window"].encode()), m)
        assert got == ggo.kmer_code(ggo.encode(w["kept"].encode()), GOLD["weight"])


def test_paper_mask_index_size(ggo):
    # one posting per whole 18-base window: 4e9 / 18 = 222 M; 8 B per posting plus
    # 16 B per list head of the 4^11 lists, in binary megabytes
    n = GOLD["bank_bases"] // GOLD["span"]
    assert n // 10**6 == GOLD["sub_sequences_millions"]
    mib = (n * 8 + 4 ** GOLD["weight"] * 16) / 2**20
    assert abs(mib - GOLD["index_megabytes"]) < 0.005 * GOLD["index_megabytes"]
    db = synth.random_db(3, n_seqs=60, lmin=0, lmax=500)
    ix = ggo.Index(db.seqs, db.off, mask=GOLD["paper_mask"])
    assert ix.n_post == sum(int(n) // 18 for n in np.diff(db.off))
    assert len(ix.list_off()) == 4 ** 11 + 1
    seq, pos = ix.postings()
    assert np.all(pos % 18 == 0)


@pytest.mark.parametrize("k", [3, 7, 11])
def test_all_ones_mask_is_the_plain_index(ggo, k):
    db = synth.random_db(4, n_seqs=80, lmin=0, lmax=600)
    qs = synth.random_queries(4, db, n=10, lmin=20, lmax=400, frac_homolog=0.8,
                              ident_lo=0.85, ident_hi=1.0, indel_rate=0.01)
    a, b = ggo.Index(db.seqs, db.off, k), ggo.Index(db.seqs, db.off, mask="1" * k)
    assert np.array_equal(a.list_off(), b.list_off())
    for x, y in zip(a.postings(), b.postings()):
        assert np.array_equal(x, y)
    prm = ggo.params(10, max_gap=2 * k, min_hsp_len=2 * k)
    for i in range(qs.n):
        ra, rb = a.search(qs.query(i), prm), b.search(qs.query(i), prm)
        assert ra[0] == rb[0] and ra[1].tobytes() == rb[1].tobytes() and ra[3] == rb[3]


@pytest.mark.parametrize("mask", ["1101", "10011", "111010010100110111", "1"])
def test_masked_hits_brute_force(ggo, mask):
    db = synth.random_db(5, n_seqs=25, lmin=0, lmax=120)
    qs = synth.random_queries(5, db, n=6, lmin=0, lmax=80, frac_homolog=0.8,
                              ident_lo=0.9, ident_hi=1.0, indel_rate=0.0)
    ix = ggo.Index(db.seqs, db.off, mask=mask)
    m = len(mask)
    keep = [t for t, ch in enumerate(mask) if ch == "1"]
    seqs = [bytes(db.seq(s)).upper().replace(b"U", b"T") for s in range(db.n_seqs)]
    for i in range(qs.n):
        q = bytes(qs.query(i)).upper().replace(b"U", b"T")
        want = []
        for qpos in range(len(q) - m + 1):
            qk = bytes(q[qpos + t] for t in keep)
            for s, sq in enumerate(seqs):
                for dpos in range(0, len(sq) - m + 1, m):
                    if bytes(sq[dpos + t] for t in keep) == qk:
                        want.append((s, dpos - qpos, qpos))
        h = ix.hits(ggo.encode(q))
        assert sorted(want) == sorted(zip(h["seq"].tolist(), h["diag"].tolist(),
                                          h["qpos"].tolist()))


def test_masked_exact_copy_found_whole(ggo):
    db = synth.small_db(n_seqs=200)
    ix = ggo.Index(db.seqs, db.off, mask=GOLD["paper_mask"])
    src = next(s for s in range(db.n_seqs) if len(db.seq(s)) >= 700)
    q = bytes(db.seq(src)[100:700])
    rc, h, n, st = ix.search(q, ggo.params(5))
    assert rc == 0 and n >= 1
    top = h[0]
    assert (int(top["seq_id"]), int(top["score"])) == (src, 600)
    assert (int(top["q_start"]), int(top["q_end"]), int(top["d_start"]), int(top["d_end"])) == \
        (0, 600, 100, 700)
    assert int(top["band_d0"]) == 100  # every run of the copy lies on diagonal 100


def test_bad_masks(ggo):
    db = synth.random_db(6, n_seqs=5, lmin=10, lmax=50)
    for bad in ["", "0000", "12", "1" * 17, "1" + "0" * 40 + "1"]:
        with pytest.raises(ValueError):
            ggo.Index(db.seqs, db.off, mask=bad)
