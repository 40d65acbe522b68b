"""GPU parity of the two index options against the oracle, bit-exact: both strands
(every sequence's reverse complement indexed as sequence n + s) and the repeat
cutoff (lists longer than max_posting dropped), alone, together and with a
spaced-seed mask, under every grouping, in pieces, in the graph-replayed and
served forms.
"""
import numpy as np
import pytest

from paper_1507_02987_amd import synth

pytestmark = pytest.mark.gpu

FIELDS = ("n_kmers", "n_hits", "n_cands", "n_merged", "n_selected", "n_cells", "n_out")
COMP = bytes.maketrans(b"ACGTUacgtu", b"TGCAAtgcaa")


def gpu():
    from paper_1507_02987_amd import gg

    gg.lib()  # fails loudly when the library is not built
    return gg


def as_rows(a):
    return [tuple(int(x) for x in r) for r in a.tolist()]


def oracle_all(oix, qs, prm_o, cap=100000):
    res, stats = [], []
    for i in range(qs.n):
        rc, h, n, st = oix.search(qs.query(i), prm_o, cap=cap)
        assert rc == 0
        res.append(h)
        stats.append(st)
    return res, stats


def check_batch(G, gix, qs, prm, want, wst, cap=100000, stats=True):
    rc, got, n, st = gix.search_batch(qs.buf, qs.off, prm, cap=cap, stats=stats)
    assert rc == 0, G.STATUS[rc]
    for i in range(qs.n):
        if stats:  # the first stage whose count differs names the stage at fault
            for f in FIELDS:
                assert int(st[i][f]) == wst[i][f], (i, f, int(st[i][f]), wst[i][f])
        assert as_rows(got[i]) == as_rows(want[i]), f"query {i}"


def flip_half(qs):
    """Every other query replaced by its reverse complement (reverse-strand homologs)."""
    parts = [bytes(qs.query(i)) for i in range(qs.n)]
    parts = [p.translate(COMP)[::-1] if i % 2 else p for i, p in enumerate(parts)]
    off = np.zeros(len(parts) + 1, np.int64)
    np.cumsum([len(p) for p in parts], out=off[1:])
    buf = np.frombuffer(b"".join(parts), np.uint8).copy()
    return synth.QuerySet(buf, off, qs.kind, qs.src_seq, qs.src_start, qs.src_end, qs.identity)


def cutoff_at(ggo, db, k, mask=None, strands=1, pct=90):
    """A cutoff at the given percentile of the non-empty list lengths, so that the
    longest lists (the repeats) are dropped and most lists kept."""
    lens = np.diff(ggo.Index(db.seqs, db.off, k, mask=mask, strands=strands).list_off())
    return max(1, int(np.percentile(lens[lens > 0], pct)))


@pytest.mark.parametrize("k,mask,strands,pct", [
    (11, None, 1, 0), (6, None, 1, 0), (0, "111010010100110111", 1, 0), (8, None, 2, 0),
    (6, None, 1, 90), (11, None, 1, 10), (6, None, 2, 90), (0, "1101011", 2, 80)])
def test_index_export_matches_oracle(ggo, k, mask, strands, pct):
    """The GPU-built index, copied back, equals the oracle's list heads and postings."""
    G = gpu()
    db = synth.repeat_db(40 + k, n_seqs=150, lmin=0, lmax=2500)
    cut = cutoff_at(ggo, db, k, mask, strands, pct) if pct else 0
    kw = dict(mask=mask, strands=strands, max_posting=cut)
    oix, gix = ggo.Index(db.seqs, db.off, k, **kw), G.Index(db.seqs, db.off, k, **kw)
    heads, post = gix.export()
    want_heads = oix.list_off()
    assert len(heads) == len(want_heads)
    bad = np.nonzero(heads.astype(np.int64) != want_heads)[0]
    assert bad.size == 0, ("heads", bad[:5], heads[bad[:5]], want_heads[bad[:5]])
    seq, pos = oix.postings()
    bad = np.nonzero((post[:, 0] != seq) | (post[:, 1] != pos))[0]
    assert bad.size == 0, ("postings", bad[:5], post[bad[:5]], seq[bad[:5]], pos[bad[:5]])


@pytest.mark.parametrize("k,mask,cut,seed", [
    (11, None, False, 41), (8, None, False, 42), (0, "111010010100110111", False, 43),
    (6, None, True, 44), (0, "1101011", True, 45)])
def test_both_strands(ggo, monkeypatch, k, mask, cut, seed):
    G = gpu()
    db = synth.repeat_db(seed, n_seqs=200, lmin=0, lmax=2500) if cut else \
        synth.random_db(seed, n_seqs=300, lmin=0, lmax=3000)
    qs = flip_half(synth.random_queries(seed, db, n=40, lmin=0, lmax=1500, frac_homolog=0.8,
                                        ident_lo=0.8, ident_hi=1.0, indel_rate=0.02))
    max_posting = cutoff_at(ggo, db, k, mask, 2) if cut else 0
    kw = dict(mask=mask, strands=2, max_posting=max_posting)
    oix, gix = ggo.Index(db.seqs, db.off, k, **kw), G.Index(db.seqs, db.off, k, **kw)
    info = gix.info()
    assert info["n_postings"] == oix.n_post and info["n_seqs"] == 2 * db.n_seqs
    assert info["n_bases"] == 2 * db.total_bp
    span = len(mask) if mask else k
    want, wst = oracle_all(oix, qs, ggo.params(20, max_gap=2 * span, min_hsp_len=2 * span))
    assert any(int(h["seq_id"]) >= db.n_seqs for w in want for h in w)  # reverse-strand hits
    for grouping in ("sort", "bucket", "probe"):
        monkeypatch.setenv("GG_GROUPING", grouping)
        check_batch(G, gix, qs, G.params(20, max_gap=2 * span, min_hsp_len=2 * span), want, wst)


@pytest.mark.parametrize("k,pct", [(6, 90), (8, 50), (11, 10)])
def test_repeat_cutoff(ggo, monkeypatch, k, pct):
    G = gpu()
    db = synth.repeat_db(46 + k, n_seqs=300, lmin=0, lmax=3000)
    cut = cutoff_at(ggo, db, k, pct=pct)
    qs = synth.random_queries(46 + k, db, n=40, lmin=0, lmax=1500, frac_homolog=0.8,
                              ident_lo=0.8, ident_hi=1.0, indel_rate=0.02)
    oix = ggo.Index(db.seqs, db.off, k, max_posting=cut)
    gix = G.Index(db.seqs, db.off, k, max_posting=cut)
    full = ggo.Index(db.seqs, db.off, k)
    assert gix.info()["n_postings"] == oix.n_post < full.n_post
    want, wst = oracle_all(oix, qs, ggo.params(20, max_gap=2 * k, min_hsp_len=2 * k))
    for grouping in ("sort", "bucket", "probe"):
        monkeypatch.setenv("GG_GROUPING", grouping)
        check_batch(G, gix, qs, G.params(20, max_gap=2 * k, min_hsp_len=2 * k), want, wst)
    # a cutoff at the longest list keeps everything
    top = int(np.diff(full.list_off()).max())
    same = G.Index(db.seqs, db.off, k, max_posting=top)
    assert same.info()["n_postings"] == full.n_post


def test_options_on_the_bank_workload(ggo, monkeypatch):
    """Both strands with a cutoff on the bank-like generator (many tiles per query),
    whole, in sequence-range pieces (the ranges cover both strands' ids), in the
    graph-replayed form and in the served form."""
    G = gpu()
    monkeypatch.setenv("GG_GROUPING", "sort")
    monkeypatch.delenv("GG_GRAPH", raising=False)
    db = synth.mid_db(n_seqs=20_000)
    qs = flip_half(synth.mid_queries(db, n=60))
    kw = dict(strands=2, max_posting=40)
    oix, gix = ggo.Index(db.seqs, db.off, 11, **kw), G.Index(db.seqs, db.off, 11, **kw)
    want, wst = oracle_all(oix, qs, ggo.params(50))
    prm = G.params(50)
    check_batch(G, gix, qs, prm, want, wst)
    hits = max(int(s["n_hits"]) for s in wst)
    gix.set_hit_budget(16 * (hits // 5))
    check_batch(G, gix, qs, prm, want, wst)
    gix.set_hit_budget(0)
    gix.profile(True)
    check_batch(G, gix, qs, prm, want, wst, cap=1000, stats=False)
    assert gix.profile_read("graph")["units"] >= 1
    gix.profile(False)
    sv = G.Server(gix, prm, max_slots=8)
    try:
        tickets = [sv.submit(qs.query(i)) for i in range(qs.n)]
        for i, t in enumerate(tickets):
            rc, h, n = sv.poll(t, cap=1000, timeout_us=-1)
            assert rc == 0 and as_rows(h) == as_rows(want[i])
    finally:
        sv.close()


def test_bad_options_rejected():
    G = gpu()
    db = synth.random_db(6, n_seqs=5, lmin=10, lmax=50)
    for kw in (dict(strands=0), dict(strands=3), dict(max_posting=-1),
               dict(strands=2, mask="0000")):
        with pytest.raises(G.GGError):
            G.Index(db.seqs, db.off, 5, **kw)
    bad = db.seqs.copy()
    bad[3] = ord("N")
    with pytest.raises(G.GGError):
        G.Index(bad, db.off, 5, strands=2)
