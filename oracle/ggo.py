"""ctypes front end of the C oracle (``ggo.c``).

TEST INFRASTRUCTURE ONLY: the oracle defines what the search must return.  Only
the test suite, the smoke check and the benchmark's CPU-baseline leg use it.  It
imports nothing from the GPU package and the GPU package never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libggo.so")
SRC = os.path.join(HERE, "ggo.c")

HIT_FIELDS = ["seq_id", "score", "q_start", "q_end", "d_start", "d_end",
              "box_q_start", "box_q_end", "box_d_start", "box_d_end", "box_len",
              "band_d0"]
HIT_DTYPE = np.dtype([(f, np.int32) for f in HIT_FIELDS])
HITREC_DTYPE = np.dtype([("seq", np.int32), ("diag", np.int32), ("qpos", np.int32)])
CAND_DTYPE = np.dtype([("seq", np.int32), ("diag", np.int32), ("qs", np.int32), ("qe", np.int32)])
BOX_DTYPE = np.dtype([(f, np.int32) for f in ("seq", "qs", "qe", "ds", "de", "dmin", "dmax")])
STATS_FIELDS = ["n_kmers", "n_hits", "n_cands", "n_merged", "n_selected", "n_cells", "n_out"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into oracle/libggo.so."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
                               SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Params(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("match", "mismatch", "gap_open", "gap_extend", "band",
                                         "xdrop", "max_gap", "min_hsp_len", "max_hits")]


def params(max_hits: int = 20, match: int = 1, mismatch: int = 3, gap_open: int = 5,
           gap_extend: int = 2, band: int = 32, xdrop: int = 20, max_gap: int = 22,
           min_hsp_len: int = 22) -> Params:
    return Params(match, mismatch, gap_open, gap_extend, band, xdrop, max_gap, min_hsp_len,
                  max_hits)


class _Index(C.Structure):
    _fields_ = [("k", C.c_int32), ("n_seqs", C.c_int64), ("seq_off", C.POINTER(C.c_int64)),
                ("base", C.POINTER(C.c_uint8)), ("n_lists", C.c_int64),
                ("list_off", C.POINTER(C.c_int64)), ("post_seq", C.POINTER(C.c_int32)),
                ("post_pos", C.POINTER(C.c_int32)), ("n_post", C.c_int64),
                ("span", C.c_int32), ("mask", C.c_uint32), ("strands", C.c_int32)]


class _Stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in STATS_FIELDS]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        P32, P64 = C.POINTER(C.c_int32), C.POINTER(C.c_int64)
        L.ggo_base_code.argtypes = [i32]
        L.ggo_base_code.restype = i32
        L.ggo_encode.argtypes = [vp, i64, vp]
        L.ggo_encode.restype = i32
        L.ggo_kmer_code.argtypes = [vp, i32]
        L.ggo_kmer_code.restype = C.c_uint32
        L.ggo_index_build.argtypes = [vp, vp, i64, i32, C.POINTER(C.POINTER(_Index))]
        L.ggo_index_build.restype = i32
        L.ggo_index_build_masked.argtypes = [vp, vp, i64, C.c_char_p,
                                             C.POINTER(C.POINTER(_Index))]
        L.ggo_index_build_masked.restype = i32
        L.ggo_index_build_opts.argtypes = [vp, vp, i64, i32, C.c_char_p, i32, i64,
                                           C.POINTER(C.POINTER(_Index))]
        L.ggo_index_build_opts.restype = i32
        L.ggo_karlin_altschul.argtypes = [i32, i32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                          C.POINTER(C.c_double)]
        L.ggo_karlin_altschul.restype = i32
        L.ggo_significance.argtypes = [i32, i64, i64, C.c_double, C.c_double,
                                       C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.ggo_significance.restype = None
        L.ggo_traceback.argtypes = [C.POINTER(_Index), vp, i64, C.POINTER(Params), vp, vp, i64,
                                    C.POINTER(i64)]
        L.ggo_traceback.restype = i32
        L.ggo_masked_code.argtypes = [vp, i32, C.c_uint32]
        L.ggo_masked_code.restype = C.c_uint32
        L.ggo_index_free.argtypes = [C.POINTER(_Index)]
        L.ggo_hits.argtypes = [C.POINTER(_Index), vp, i32, C.POINTER(vp), P64]
        L.ggo_hits.restype = i32
        L.ggo_group.argtypes = [vp, i64]
        L.ggo_chain.argtypes = [vp, i64, i32, i32, i32, C.POINTER(vp), P64]
        L.ggo_chain.restype = i32
        L.ggo_extend.argtypes = [vp, i32, vp, i32, vp, C.POINTER(Params), vp]
        L.ggo_merge.argtypes = [vp, i64, C.POINTER(vp), P64]
        L.ggo_merge.restype = i32
        L.ggo_select.argtypes = [vp, i64, i32, C.POINTER(vp), P64]
        L.ggo_select.restype = i32
        L.ggo_bsw.argtypes = [vp, vp, vp, C.POINTER(Params), vp]
        L.ggo_bsw.restype = i64
        L.ggo_report.argtypes = [vp, i64]
        L.ggo_report.restype = i64
        L.ggo_search.argtypes = [C.POINTER(_Index), vp, i64, C.POINTER(Params), vp, i32, P32,
                                 C.POINTER(_Stats)]
        L.ggo_search.restype = i32
        L.ggo_free.argtypes = [vp]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _take(ptr: C.c_void_p, n: int, dtype) -> np.ndarray:
    """Copy n records from a malloc'd C array and free it."""
    if n:
        out = np.frombuffer((C.c_char * (n * dtype.itemsize)).from_address(ptr.value),
                            dtype=dtype).copy()
    else:
        out = np.zeros(0, dtype=dtype)
    lib().ggo_free(ptr)
    return out


def encode(s: bytes | np.ndarray) -> np.ndarray:
    """O0: 2-bit codes; raises ValueError outside the alphabet."""
    a = np.frombuffer(bytes(s), dtype=np.uint8) if not isinstance(s, np.ndarray) else s
    a = np.ascontiguousarray(a, dtype=np.uint8)
    out = np.empty(max(len(a), 1), dtype=np.uint8)
    if lib().ggo_encode(_ptr(a), len(a), _ptr(out)) != 0:
        raise ValueError("byte outside the nucleotide alphabet")
    return out[: len(a)]


def kmer_code(codes: np.ndarray, k: int) -> int:
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    assert len(codes) >= k
    return int(lib().ggo_kmer_code(_ptr(codes), k))


def karlin_altschul(match: int = 1, mismatch: int = 3) -> tuple[float, float, float]:
    """(lambda, K, H) of ungapped +match / -mismatch scoring on uniform bases."""
    lam, K, H = C.c_double(), C.c_double(), C.c_double()
    if lib().ggo_karlin_altschul(match, mismatch, C.byref(lam), C.byref(K), C.byref(H)) != 0:
        raise ValueError("scores must be positive")
    return lam.value, K.value, H.value


def significance(score: int, m: int, n: int, lam: float, K: float) -> tuple[float, float]:
    """(bit score, e-value) of a score for a query of m bases against n bank bases."""
    bits, ev = C.c_double(), C.c_double()
    lib().ggo_significance(score, m, n, lam, K, C.byref(bits), C.byref(ev))
    return bits.value, ev.value


def mask_bits(mask: str) -> int:
    """Bit t set when the mask keeps the window's base t."""
    return sum(1 << t for t, ch in enumerate(mask) if ch == "1")


def masked_code(codes: np.ndarray, mask: str) -> int:
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    assert len(codes) >= len(mask)
    return int(lib().ggo_masked_code(_ptr(codes), len(mask), mask_bits(mask)))


class Index:
    """O1: the formatted data bank and its inverted index, owned by the C side.
    k windows, or windows of a mask's length coded on its '1' positions; strands=2
    adds every sequence's reverse complement (as sequence n + s); max_posting > 0
    drops the lists longer than it."""

    def __init__(self, seqs: np.ndarray, off: np.ndarray, k: int = 0, mask: str | None = None,
                 strands: int = 1, max_posting: int = 0):
        self._seqs = np.ascontiguousarray(seqs, dtype=np.uint8)
        self._off = np.ascontiguousarray(off, dtype=np.int64)
        p = C.POINTER(_Index)()
        if strands != 1 or max_posting != 0:
            rc = lib().ggo_index_build_opts(_ptr(self._seqs), _ptr(self._off), len(self._off) - 1,
                                            k, mask.encode() if mask is not None else None,
                                            strands, max_posting, C.byref(p))
        elif mask is not None:
            rc = lib().ggo_index_build_masked(_ptr(self._seqs), _ptr(self._off),
                                              len(self._off) - 1, mask.encode(), C.byref(p))
        else:
            rc = lib().ggo_index_build(_ptr(self._seqs), _ptr(self._off), len(self._off) - 1, k,
                                       C.byref(p))
        if rc != 0:
            raise ValueError(f"ggo_index_build failed with status {rc}")
        self._p = p
        self.k = int(p.contents.k)
        self.span = int(p.contents.span)
        self.mask = mask
        self.strands = int(p.contents.strands)
        self.n_seqs = int(p.contents.n_seqs)

    def __del__(self):
        if getattr(self, "_p", None):
            lib().ggo_index_free(self._p)
            self._p = None

    @property
    def n_post(self) -> int:
        return int(self._p.contents.n_post)

    def list_off(self) -> np.ndarray:
        ix = self._p.contents
        return np.ctypeslib.as_array(ix.list_off, shape=(ix.n_lists + 1,)).copy()

    def postings(self) -> tuple[np.ndarray, np.ndarray]:
        ix = self._p.contents
        n = ix.n_post
        if n == 0:
            return np.zeros(0, np.int32), np.zeros(0, np.int32)
        return (np.ctypeslib.as_array(ix.post_seq, shape=(n,)).copy(),
                np.ctypeslib.as_array(ix.post_pos, shape=(n,)).copy())

    def seq_codes(self, s: int) -> np.ndarray:
        ix = self._p.contents
        lo, hi = ix.seq_off[s], ix.seq_off[s + 1]
        if hi == lo:
            return np.zeros(0, np.uint8)
        return np.ctypeslib.as_array(ix.base, shape=(ix.seq_off[ix.n_seqs],))[lo:hi].copy()

    # ---- stages
    def hits(self, qcodes: np.ndarray) -> np.ndarray:
        q = np.ascontiguousarray(qcodes, dtype=np.uint8)
        p, n = C.c_void_p(), C.c_int64()
        rc = lib().ggo_hits(self._p, _ptr(q), len(q), C.byref(p), C.byref(n))
        if rc != 0:
            raise MemoryError(rc)
        if not p.value:
            return np.zeros(0, HITREC_DTYPE)
        return _take(p, n.value, HITREC_DTYPE)

    def traceback(self, query: bytes | np.ndarray, prm: Params, hit) -> str:
        """The path of one reported hit as '=' 'X' 'I' 'D' operations, first to last."""
        q = np.frombuffer(bytes(query), np.uint8) if not isinstance(query, np.ndarray) else query
        q = np.ascontiguousarray(q, dtype=np.uint8)
        h = np.ascontiguousarray(np.array(hit, dtype=HIT_DTYPE).reshape(1))
        cap = int(h["q_end"][0] - h["q_start"][0] + h["d_end"][0] - h["d_start"][0]) + 1
        buf = C.create_string_buffer(max(cap, 1))
        n = C.c_int64()
        rc = lib().ggo_traceback(self._p, _ptr(q), len(q), C.byref(prm), _ptr(h), buf, cap,
                                 C.byref(n))
        if rc != 0:
            raise ValueError(f"ggo_traceback failed with status {rc}")
        return buf.raw[:n.value].decode()

    def search(self, query: bytes | np.ndarray, prm: Params, cap: int = 1 << 16):
        q = np.frombuffer(bytes(query), np.uint8) if not isinstance(query, np.ndarray) else query
        q = np.ascontiguousarray(q, dtype=np.uint8)
        out = np.zeros(max(cap, 1), dtype=HIT_DTYPE)
        n = C.c_int32()
        st = _Stats()
        rc = lib().ggo_search(self._p, _ptr(q), len(q), C.byref(prm), _ptr(out), cap, C.byref(n),
                              C.byref(st))
        stats = {f: int(getattr(st, f)) for f in STATS_FIELDS}
        return rc, out[: min(n.value, cap)].copy(), n.value, stats


def group(h: np.ndarray) -> np.ndarray:
    h = np.ascontiguousarray(h.copy(), dtype=HITREC_DTYPE)
    lib().ggo_group(_ptr(h), len(h))
    return h


def chain(h: np.ndarray, k: int, max_gap: int, min_len: int) -> np.ndarray:
    h = np.ascontiguousarray(h, dtype=HITREC_DTYPE)
    p, n = C.c_void_p(), C.c_int64()
    rc = lib().ggo_chain(_ptr(h), len(h), k, max_gap, min_len, C.byref(p), C.byref(n))
    assert rc == 0
    return _take(p, n.value, CAND_DTYPE)


def extend(qcodes: np.ndarray, scodes: np.ndarray, cand, prm: Params) -> np.ndarray:
    q = np.ascontiguousarray(qcodes, dtype=np.uint8)
    s = np.ascontiguousarray(scodes, dtype=np.uint8)
    c = np.array([tuple(cand)], dtype=CAND_DTYPE)
    out = np.zeros(1, dtype=BOX_DTYPE)
    lib().ggo_extend(_ptr(q), len(q), _ptr(s), len(s), _ptr(c), C.byref(prm), _ptr(out))
    return out[0]


def merge(boxes: np.ndarray) -> np.ndarray:
    b = np.ascontiguousarray(boxes, dtype=BOX_DTYPE)
    p, n = C.c_void_p(), C.c_int64()
    assert lib().ggo_merge(_ptr(b), len(b), C.byref(p), C.byref(n)) == 0
    return _take(p, n.value, BOX_DTYPE)


def select(boxes: np.ndarray, max_hits: int) -> np.ndarray:
    b = np.ascontiguousarray(boxes, dtype=BOX_DTYPE)
    p, n = C.c_void_p(), C.c_int64()
    assert lib().ggo_select(_ptr(b), len(b), max_hits, C.byref(p), C.byref(n)) == 0
    allb = _take(p, len(b), BOX_DTYPE)
    return allb[: n.value]


def bsw(qcodes: np.ndarray, scodes: np.ndarray, box, prm: Params):
    """O9 on one box; returns (hit record, in-band cell count)."""
    q = np.ascontiguousarray(qcodes, dtype=np.uint8)
    s = np.ascontiguousarray(scodes, dtype=np.uint8)
    b = np.array([tuple(box)], dtype=BOX_DTYPE)
    out = np.zeros(1, dtype=HIT_DTYPE)
    cells = lib().ggo_bsw(_ptr(q), _ptr(s), _ptr(b), C.byref(prm), _ptr(out))
    return out[0], int(cells)


def report(hits: np.ndarray) -> np.ndarray:
    h = np.ascontiguousarray(hits.copy(), dtype=HIT_DTYPE)
    m = lib().ggo_report(_ptr(h), len(h))
    return h[:m]
