"""Saved and loaded indexes (Section 2.1: the index is kept on disk and read whole
at start) serve exactly as the index they were saved from: the same list heads,
postings and counts, and bit-identical searches, for plain, masked, two-strand
and cut builds; a damaged file is refused."""
import numpy as np
import pytest

from paper_1507_02987_amd import synth

pytestmark = pytest.mark.gpu


def gpu():
    from paper_1507_02987_amd import gg

    gg.lib()  # fails loudly when the library is not built
    return gg


@pytest.mark.parametrize("k,kw", [(11, {}), (0, dict(mask="111010010100110111")),
                                  (8, dict(strands=2, max_posting=3))])
def test_save_load_round_trip(ggo, tmp_path, k, kw):
    G = gpu()
    db = synth.random_db(61, n_seqs=300, lmin=0, lmax=3000)
    qs = synth.random_queries(61, db, n=40, lmin=0, lmax=1500, frac_homolog=0.8,
                              ident_lo=0.8, ident_hi=1.0, indel_rate=0.02)
    a = G.Index(db.seqs, db.off, k, **kw)
    path = tmp_path / "bank.ggi"
    a.save(str(path))
    b = G.Index.load(str(path))
    assert a.info() == b.info()
    ha, pa = a.export()
    hb, pb = b.export()
    assert np.array_equal(ha, hb) and np.array_equal(pa, pb)
    prm = G.params(20)
    ra = a.search_batch(qs.buf, qs.off, prm, cap=1000, stats=True)
    rb = b.search_batch(qs.buf, qs.off, prm, cap=1000, stats=True)
    assert ra[0] == rb[0] == 0
    assert sum(len(x) for x in ra[1]) > 0
    for i in range(qs.n):
        assert ra[1][i].tobytes() == rb[1][i].tobytes()
        assert ra[3][i].tobytes() == rb[3][i].tobytes()
    # the loaded index against the oracle built from the sequences
    oix = ggo.Index(db.seqs, db.off, k, **kw)
    for i in range(0, qs.n, 5):
        orc, oh, on, _ = oix.search(qs.query(i), ggo.params(20), cap=1000)
        assert [tuple(r) for r in rb[1][i].tolist()] == [tuple(r) for r in oh.tolist()]


def test_damaged_file_refused(tmp_path):
    G = gpu()
    db = synth.random_db(62, n_seqs=50, lmin=0, lmax=500)
    a = G.Index(db.seqs, db.off, 9)
    path = tmp_path / "bank.ggi"
    a.save(str(path))
    raw = bytearray(path.read_bytes())
    raw[len(raw) // 2] ^= 0x10
    bad = tmp_path / "bad.ggi"
    bad.write_bytes(bytes(raw))
    with pytest.raises(G.GGError) as e:
        G.Index.load(str(bad))
    assert e.value.status == G.GG_EIO
    with pytest.raises(G.GGError):
        G.Index.load(str(tmp_path / "missing.ggi"))
