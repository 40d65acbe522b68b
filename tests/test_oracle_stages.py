"""Pins for the oracle's hit retrieval (O3), grouping and chaining (O4/O5),
extension (O6), merging (O7), selection (O8) and report order (O10).

Pinned against brute-force substring comparison, the hand-worked cases in
tests/golden (Section 2.2), and hand-built record arrays whose expected results
follow from the definitions by inspection.
"""
import json
import os

import numpy as np
import pytest

from paper_1507_02987_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
LETTERS = "ACGT"


def codes_of(text: str) -> np.ndarray:
    return np.array(["ACGT".index(c) for c in text], dtype=np.uint8)


# ------------------------------------------------------------------ O3

@pytest.mark.parametrize("k,seed", [(4, 0), (6, 1), (11, 2)])
def test_hits_equal_brute_force(ggo, k, seed):
    db = synth.random_db(seed, n_seqs=30, lmin=5, lmax=400)
    rng = np.random.default_rng(seed)
    ix = ggo.Index(db.seqs, db.off, k)
    text = [db.seq(s).tobytes().decode() for s in range(db.n_seqs)]
    for _ in range(5):
        # half the query copied from the bank so that long k always has hits
        s0 = int(rng.integers(db.n_seqs))
        q = text[s0][: 60] + "".join(rng.choice(list(LETTERS), size=60))
        got = ix.hits(codes_of(q))
        want = set()
        for s, seq in enumerate(text):
            for w in range(len(seq) // k):
                kmer = seq[w * k:(w + 1) * k]
                for qpos in range(len(q) - k + 1):
                    if q[qpos:qpos + k] == kmer:
                        want.add((s, w * k - qpos, qpos))
        assert len(got) == len(want)
        assert set(map(tuple, got.tolist())) == want
        # generation order: query offset major
        assert np.all(np.diff(got["qpos"]) >= 0)


def test_short_query_has_no_hits(ggo):
    db = synth.random_db(3, 5, 50, 60)
    ix = ggo.Index(db.seqs, db.off, 11)
    assert len(ix.hits(codes_of("ACGTACGTAC"))) == 0


# ------------------------------------------------------------------ O4/O5

def hits_array(rows):
    return np.array([tuple(r) for r in rows], dtype=np.dtype([("seq", np.int32),
                                                              ("diag", np.int32),
                                                              ("qpos", np.int32)]))


def test_group_order(ggo):
    rows = [(2, 5, 40), (1, 7, 3), (2, -3, 90), (1, 7, 0), (0, 100, 11), (2, 5, 18)]
    got = ggo.group(hits_array(rows))
    assert [tuple(r) for r in got.tolist()] == sorted(rows)


def test_chain_gap_threshold(ggo):
    k, G = 11, 22
    # qpos 0 and 33: gap 33 - (0 + 11) = 22 <= G joins; 33 and 67: gap 23 > G splits
    h = hits_array([(1, 5, 0), (1, 5, 33), (1, 5, 67), (1, 5, 78)])
    got = ggo.chain(h, k, G, 22)
    assert [tuple(r) for r in got.tolist()] == [(1, 5, 0, 44), (1, 5, 67, 89)]


def test_chain_min_length(ggo):
    k = 11
    h = hits_array([(1, 0, 0), (1, 0, 11), (2, 0, 0), (3, 4, 50)])
    assert [tuple(r) for r in ggo.chain(h, k, 22, 22).tolist()] == [(1, 0, 0, 22)]
    assert [tuple(r) for r in ggo.chain(h, k, 22, 23).tolist()] == []
    # M <= k keeps single hits too
    assert len(ggo.chain(h, k, 22, 11)) == 3


def test_chain_never_crosses_groups(ggo):
    k = 11
    h = hits_array([(1, 0, 0), (1, 1, 11), (2, 1, 22), (2, 1, 33)])
    got = ggo.chain(h, k, 100, 1)
    assert [tuple(r) for r in got.tolist()] == [(1, 0, 0, 11), (1, 1, 11, 22), (2, 1, 22, 44)]


def test_exact_copy_case(ggo):
    """tests/golden/chain_extend.json: query = S[100:300) of one sequence."""
    g = json.load(open(os.path.join(GOLD, "chain_extend.json")))["exact_copy_case"]
    k = g["k"]
    rng = np.random.default_rng(11)
    S = "".join(rng.choice(list(LETTERS), size=400))
    other = "".join(rng.choice(list(LETTERS), size=300))
    seqs = np.frombuffer((other + S).encode(), np.uint8)
    off = np.array([0, 300, 700], np.int64)
    ix = ggo.Index(seqs, off, k)
    q = S[g["src_start"]:g["src_start"] + g["L"]]
    hits = ggo.group(ix.hits(codes_of(q)))
    on = hits[(hits["seq"] == 1) & (hits["diag"] == g["diag"])]
    assert len(on) == g["n_hits_on_diag"]
    assert on["qpos"][0] == g["first_qpos"] and on["qpos"][-1] == g["last_qpos"]
    cands = ggo.chain(hits, k, 22, 22)
    mine = cands[(cands["seq"] == 1) & (cands["diag"] == g["diag"])]
    assert [(int(c["qs"]), int(c["qe"])) for c in mine] == [tuple(g["run"])]
    prm = ggo.params(20)
    box = ggo.extend(codes_of(q), codes_of(S), mine[0], prm)
    assert (box["qs"], box["qe"], box["ds"], box["de"]) == tuple(g["box"])
    rc, res, n, st = ix.search(q.encode(), prm)
    assert rc == 0 and n >= 1
    top = res[0]
    assert (top["seq_id"], top["score"]) == (1, g["score"])
    assert (top["q_start"], top["q_end"], top["d_start"], top["d_end"]) == tuple(g["box"])


# ------------------------------------------------------------------ O6

def build_pattern(pattern, rng):
    """Query and database letters that realise a run-length match pattern."""
    qa, sa = [], []
    for letter, count in pattern:
        for _ in range(count):
            a = int(rng.integers(4))
            qa.append(a)
            sa.append(a if letter == "M" else (a + 1 + int(rng.integers(3))) % 4)
    return qa, sa


@pytest.mark.parametrize("side", ["right", "left"])
def test_xdrop_cases(ggo, side):
    g = json.load(open(os.path.join(GOLD, "chain_extend.json")))["xdrop_cases"]
    rng = np.random.default_rng(5)
    prm = ggo.params(20)
    for case in g["cases"]:
        pq, ps = build_pattern(case["pattern"], rng)
        seed = [int(x) for x in rng.integers(0, 4, size=22)]
        if side == "right":
            q = seed + pq
            s = seed + ps
            cand = (0, 0, 0, 22)
        else:
            q = pq[::-1] + seed
            s = ps[::-1] + seed
            cand = (0, 0, len(pq), len(pq) + 22)
        box = ggo.extend(np.array(q, np.uint8), np.array(s, np.uint8), cand, prm)
        ext = (box["qe"] - cand[3]) if side == "right" else (cand[2] - box["qs"])
        assert ext == case["ext"], case["why"]
        other = (cand[2] - box["qs"]) if side == "right" else (box["qe"] - cand[3])
        assert other == 0
        assert box["ds"] - box["qs"] == 0 and box["de"] - box["qe"] == 0
        assert box["dmin"] == box["dmax"] == 0


def test_xdrop_stops_at_sequence_ends(ggo):
    prm = ggo.params(20)
    q = np.zeros(50, np.uint8)
    s = np.zeros(40, np.uint8)
    # diagonal d = -10: database ends first on the right, query start first on the left
    box = ggo.extend(q, s, (0, -10, 20, 42), prm)
    assert (box["qs"], box["qe"], box["ds"], box["de"]) == (10, 50, 0, 40)
    box = ggo.extend(q, s, (0, 5, 20, 30), prm)
    assert (box["qs"], box["qe"], box["ds"], box["de"]) == (0, 35, 5, 40)


# ------------------------------------------------------------------ O7/O8

def boxes(rows):
    return np.array([tuple(r) for r in rows], dtype=np.dtype([(f, np.int32) for f in (
        "seq", "qs", "qe", "ds", "de", "dmin", "dmax")]))


def test_merge_cases(ggo):
    g = json.load(open(os.path.join(GOLD, "merge_select.json")))
    for case in g["merge_cases"]:
        got = ggo.merge(boxes(case["in"]))
        assert [list(r) for r in got.tolist()] == case["out"], case["about"]


def test_select_case(ggo):
    g = json.load(open(os.path.join(GOLD, "merge_select.json")))["select_case"]
    got = ggo.select(boxes(g["in"]), 0)
    assert [list(r) for r in got.tolist()] == g["order"]
    lens = np.minimum(got["qe"] - got["qs"], got["de"] - got["ds"])
    assert lens.tolist() == g["lengths"]
    assert [list(r) for r in ggo.select(boxes(g["in"]), 2).tolist()] == g["order"][:2]
    assert len(ggo.select(boxes(g["in"]), -1)) == len(g["in"])


# ------------------------------------------------------------------ O10

def test_report_order_and_drop(ggo):
    dt = np.dtype([(f, np.int32) for f in ggo.HIT_FIELDS])
    rows = [
        (5, 10, 0, 10, 0, 10, 0, 10, 0, 10, 10, 0),
        (2, 30, 4, 40, 4, 40, 0, 50, 0, 50, 50, 0),
        (1, 30, 4, 40, 4, 40, 0, 50, 0, 50, 50, 0),
        (1, 30, 2, 40, 9, 47, 0, 50, 0, 50, 50, 7),
        (1, 0, -1, -1, -1, -1, 0, 5, 0, 5, 5, 0),
        (1, 30, 2, 40, 9, 47, 1, 50, 0, 50, 49, 7),
        (1, 30, 4, 40, 4, 40, 0, 50, 0, 50, 50, -3),  # ties rows[2] but for the band centre
    ]
    got = ggo.report(np.array(rows, dtype=dt))
    assert [tuple(r) for r in got.tolist()] == [rows[3], rows[5], rows[6], rows[2], rows[1],
                                                rows[0]]
