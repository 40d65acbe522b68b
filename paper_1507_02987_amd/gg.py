"""Python binding of libgg.so (include/gg.h): argument marshalling only.

Every stage of a search runs in the library's HIP kernels.  There is no CPU
fallback: if the compiled library is missing, importing this module works but
any call raises ``RuntimeError``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgg.so")

(GG_OK, GG_EINVAL, GG_ENOMEM, GG_EDEVICE, GG_EAGAIN, GG_ETRUNC, GG_ENOTFOUND, GG_EBUDGET, GG_EIO,
 GG_ESCRATCH) = range(10)
STATUS = {0: "GG_OK", 1: "GG_EINVAL", 2: "GG_ENOMEM", 3: "GG_EDEVICE", 4: "GG_EAGAIN",
          5: "GG_ETRUNC", 6: "GG_ENOTFOUND", 7: "GG_EBUDGET", 8: "GG_EIO", 9: "GG_ESCRATCH"}
NOALLOC_SCRATCH_BYTES = 64 << 20

HIT_FIELDS = ("seq_id", "score", "q_start", "q_end", "d_start", "d_end",
              "box_q_start", "box_q_end", "box_d_start", "box_d_end", "box_len",
              "band_d0")
HIT_DTYPE = np.dtype([(f, np.int32) for f in HIT_FIELDS])
STAT_FIELDS = ("n_kmers", "n_hits", "n_cands", "n_merged", "n_selected", "n_cells", "n_out")
STAT_DTYPE = np.dtype([(f, np.int64) for f in STAT_FIELDS])

# Exported symbols of include/gg.h, in declaration order.
SYMBOLS = ("gg_index_build", "gg_index_build_masked", "gg_index_build_ex", "gg_index_free",
           "gg_index_info", "gg_index_export", "gg_index_save", "gg_index_load",
           "gg_karlin_altschul", "gg_traceback_noalloc", "gg_hit_significance", "gg_traceback",
           "gg_index_set_hit_budget",
           "gg_index_get_tuning", "gg_index_set_tuning", "gg_index_autotune",
           "gg_search", "gg_search_batch", "gg_search_batch_device", "gg_device_alloc",
           "gg_device_free", "gg_memcpy_to_device", "gg_memcpy_to_host", "gg_device_copy",
           "gg_device_read",
           "gg_profile_enable", "gg_profile_read",
           "gg_server_create", "gg_serve_submit", "gg_serve_poll", "gg_server_info",
           "gg_server_destroy",
           "gg_strerror")


class GGError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {STATUS.get(status, status)}")
        self.status = status


class Params(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("match", "mismatch", "gap_open", "gap_extend", "band",
                                         "xdrop", "max_gap", "min_hsp_len", "max_hits")]


class IndexOptions(C.Structure):
    _fields_ = [("k", C.c_int32), ("mask", C.c_char_p), ("strands", C.c_int32),
                ("max_posting", C.c_int64)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("batches", C.c_int64),
                ("budget_bytes", C.c_uint64), ("peak_inflight_bytes", C.c_uint64),
                ("inflight_bytes", C.c_uint64), ("peak_inflight_slots", C.c_int64),
                ("inflight_slots", C.c_int64), ("peak_batch_queries", C.c_int64),
                ("over_budget", C.c_int64), ("calls_inside", C.c_int64)]


class Tuning(C.Structure):
    _fields_ = [("grouping", C.c_int32), ("lane_steps", C.c_int32), ("ms", C.c_double),
                ("wave_log2", C.c_int32), ("graph", C.c_int32), ("graph_query_log2", C.c_int32)]


GROUPINGS = ("probe", "bucket", "sort")


def karlin_altschul(match: int = 1, mismatch: int = 3) -> tuple[float, float, float]:
    """gg_karlin_altschul: (lambda, K, H) of ungapped scoring on uniform bases."""
    lam, K, H = C.c_double(), C.c_double(), C.c_double()
    rc = lib().gg_karlin_altschul(match, mismatch, C.byref(lam), C.byref(K), C.byref(H))
    if rc != GG_OK:
        raise GGError(rc, "gg_karlin_altschul")
    return lam.value, K.value, H.value


def significance(hits: np.ndarray, query_len: int, bank_bases: int, lam: float, K: float):
    """gg_hit_significance: (bit scores, e-values) of one query's hits."""
    h = np.ascontiguousarray(hits, dtype=HIT_DTYPE)
    bits = np.zeros(max(len(h), 1))
    ev = np.zeros(max(len(h), 1))
    rc = lib().gg_hit_significance(_ptr(h) if len(h) else None, len(h), query_len, bank_bases,
                                   lam, K, _ptr(bits), _ptr(ev))
    if rc != GG_OK:
        raise GGError(rc, "gg_hit_significance")
    return bits[:len(h)], ev[:len(h)]


def params(max_hits: int = 20, match: int = 1, mismatch: int = 3, gap_open: int = 5,
           gap_extend: int = 2, band: int = 32, xdrop: int = 20, max_gap: int = 22,
           min_hsp_len: int = 22) -> Params:
    """The workloads' scoring: +1/-3, gap 5 + 2 g, band 32, X-drop 20."""
    return Params(match, mismatch, gap_open, gap_extend, band, xdrop, max_gap, min_hsp_len,
                  max_hits)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_1507_02987_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
        L.gg_index_build.argtypes = [vp, vp, i64, i32, i32, C.POINTER(vp)]
        L.gg_index_build_masked.argtypes = [vp, vp, i64, C.c_char_p, i32, C.POINTER(vp)]
        L.gg_index_build_ex.argtypes = [vp, vp, i64, C.POINTER(IndexOptions), i32, C.POINTER(vp)]
        L.gg_index_export.argtypes = [vp, vp, vp, i64]
        L.gg_index_save.argtypes = [vp, C.c_char_p]
        dp = C.POINTER(C.c_double)
        L.gg_karlin_altschul.argtypes = [i32, i32, dp, dp, dp]
        L.gg_hit_significance.argtypes = [vp, i64, i64, i64, C.c_double, C.c_double, vp, vp]
        L.gg_traceback.argtypes = [vp, vp, i64, C.POINTER(Params), vp, i32, vp, i64, vp, vp]
        L.gg_traceback_noalloc.argtypes = [vp, vp, i64, C.POINTER(Params), vp, i32, vp, i64, vp,
                                           vp]
        L.gg_index_load.argtypes = [C.c_char_p, i32, C.POINTER(vp)]
        L.gg_index_free.argtypes = [vp]
        L.gg_index_free.restype = None
        L.gg_index_info.argtypes = [vp, vp, vp, vp, vp]
        L.gg_index_set_hit_budget.argtypes = [vp, u64]
        L.gg_index_get_tuning.argtypes = [vp, C.POINTER(Tuning)]
        L.gg_index_set_tuning.argtypes = [vp, C.POINTER(Tuning)]
        L.gg_index_autotune.argtypes = [vp, vp, vp, i64, C.POINTER(Params), C.POINTER(Tuning)]
        L.gg_search.argtypes = [vp, vp, i64, C.POINTER(Params), vp, i32, vp]
        L.gg_search_batch.argtypes = [vp, vp, vp, i64, C.POINTER(Params), vp, i32, vp, vp]
        L.gg_search_batch_device.argtypes = [vp, vp, vp, i64, C.POINTER(Params), vp, i32, vp, vp]
        L.gg_device_alloc.argtypes = [i32, u64, C.POINTER(vp)]
        L.gg_device_free.argtypes = [i32, vp]
        L.gg_memcpy_to_device.argtypes = [vp, vp, u64]
        L.gg_memcpy_to_host.argtypes = [vp, vp, u64]
        L.gg_device_copy.argtypes = [vp, vp, u64]
        L.gg_device_read.argtypes = [vp, u64, C.POINTER(u64)]
        L.gg_profile_enable.argtypes = [vp, i32]
        L.gg_profile_read.argtypes = [vp, C.c_char_p, vp, vp, vp]
        L.gg_server_create.argtypes = [vp, C.POINTER(Params), u64, i32, C.POINTER(vp)]
        L.gg_serve_submit.argtypes = [vp, vp, i64, vp]
        L.gg_serve_poll.argtypes = [vp, u64, vp, i32, vp, i32]
        L.gg_server_info.argtypes = [vp, C.POINTER(ServerStats)]
        L.gg_server_destroy.argtypes = [vp]
        L.gg_server_destroy.restype = None
        L.gg_strerror.argtypes = [i32]
        L.gg_strerror.restype = C.c_char_p
        for name in SYMBOLS:
            fn = getattr(L, name)
            if fn.restype is C.c_int:
                fn.restype = i32
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _u8(x) -> np.ndarray:
    if isinstance(x, np.ndarray):
        return np.ascontiguousarray(x, dtype=np.uint8)
    return np.frombuffer(bytes(x), dtype=np.uint8)


class Index:
    """gg_index_build / gg_index_free: device-resident data bank and inverted index."""

    def __init__(self, seqs, seq_off, k: int = 0, device: int = 0, mask: str | None = None,
                 strands: int = 1, max_posting: int = 0):
        """k: contiguous windows of k bases; mask: a '0'/'1' spaced-seed mask instead
        (gg_index_build_masked), whose weight is then the index's k; strands=2 and
        max_posting > 0 go through gg_index_build_ex."""
        s = _u8(seqs)
        off = np.ascontiguousarray(seq_off, dtype=np.int64)
        h = C.c_void_p()
        if strands != 1 or max_posting != 0:
            opt = IndexOptions(k, mask.encode() if mask is not None else None, strands,
                               max_posting)
            rc = lib().gg_index_build_ex(_ptr(s) if len(s) else None, _ptr(off), len(off) - 1,
                                         C.byref(opt), device, C.byref(h))
            name = "gg_index_build_ex"
            if mask is not None:
                k = mask.count("1")
        elif mask is not None:
            rc = lib().gg_index_build_masked(_ptr(s) if len(s) else None, _ptr(off), len(off) - 1,
                                             mask.encode(), device, C.byref(h))
            name = "gg_index_build_masked"
            k = mask.count("1")
        else:
            rc = lib().gg_index_build(_ptr(s) if len(s) else None, _ptr(off), len(off) - 1, k,
                                      device, C.byref(h))
            name = "gg_index_build"
        if rc != GG_OK:
            raise GGError(rc, name)
        self._h = h
        self.k = k
        self.mask = mask
        self.span = len(mask) if mask is not None else k
        self.strands = strands
        self.max_posting = max_posting

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().gg_index_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        k = C.c_int32()
        rc = lib().gg_index_info(self._h, C.byref(a), C.byref(b), C.byref(c), C.byref(k))
        if rc != GG_OK:
            raise GGError(rc, "gg_index_info")
        return {"n_postings": a.value, "n_bases": b.value, "n_seqs": c.value, "k": k.value}

    def save(self, path: str):
        """gg_index_save: the index and its 2-bit bank to a file."""
        rc = lib().gg_index_save(self._h, os.fsencode(path))
        if rc != GG_OK:
            raise GGError(rc, "gg_index_save")

    @classmethod
    def load(cls, path: str, device: int = 0) -> "Index":
        """gg_index_load: an index saved by save(), on `device`."""
        h = C.c_void_p()
        rc = lib().gg_index_load(os.fsencode(path), device, C.byref(h))
        if rc != GG_OK:
            raise GGError(rc, "gg_index_load")
        self = cls.__new__(cls)
        self._h = h
        self.k = self.info()["k"]
        self.mask = self.span = None  # not reported by the library
        self.strands = self.max_posting = None
        return self

    def export(self):
        """gg_index_export: (list heads u32[4^k + 1], postings int32[n, 2] of (seq, pos))."""
        n = self.info()["n_postings"]
        heads = np.zeros((1 << (2 * self.k)) + 1, np.uint32)
        post = np.zeros((max(n, 1), 2), np.int32)
        rc = lib().gg_index_export(self._h, _ptr(heads), _ptr(post), n)
        if rc != GG_OK:
            raise GGError(rc, "gg_index_export")
        return heads, post[:n]

    def traceback(self, query, prm: Params, hits: np.ndarray, noalloc: bool = False):
        """gg_traceback (gg_traceback_noalloc when noalloc): (status, list of
        operation strings, one per hit)."""
        q = _u8(query)
        h = np.ascontiguousarray(hits, dtype=HIT_DTYPE)
        n = len(h)
        off = np.zeros(n + 1, np.int64)
        ln = np.zeros(max(n, 1), np.int32)
        spans = (h["q_end"].astype(np.int64) - h["q_start"]) + (h["d_end"] - h["d_start"])
        cap = int(spans.clip(min=0).sum()) if n else 0
        buf = np.zeros(max(cap, 1), np.uint8)
        fn = lib().gg_traceback_noalloc if noalloc else lib().gg_traceback
        rc = fn(self._h, _ptr(q) if len(q) else None, len(q), C.byref(prm),
                _ptr(h) if n else None, n, _ptr(buf), cap, _ptr(off), _ptr(ln))
        if rc not in (GG_OK, GG_EINVAL) or (rc == GG_EINVAL and n and off[n] == 0):
            return rc, []
        return rc, [buf[off[i]:off[i] + ln[i]].tobytes().decode() for i in range(n)]

    def set_hit_budget(self, nbytes: int):
        rc = lib().gg_index_set_hit_budget(self._h, int(nbytes))
        if rc != GG_OK:
            raise GGError(rc, "gg_index_set_hit_budget")

    def tuning(self) -> dict:
        t = Tuning()
        rc = lib().gg_index_get_tuning(self._h, C.byref(t))
        if rc != GG_OK:
            raise GGError(rc, "gg_index_get_tuning")
        return {"grouping": GROUPINGS[t.grouping], "lane_steps": t.lane_steps,
                "wave_log2": t.wave_log2, "graph": t.graph, "graph_query_log2": t.graph_query_log2}

    def set_tuning(self, grouping: str = "sort", lane_steps: int = 256, wave_log2: int = 0,
                   graph: int = 1, graph_query_log2: int = 0):
        t = Tuning(GROUPINGS.index(grouping), lane_steps, 0.0, wave_log2, graph, graph_query_log2)
        rc = lib().gg_index_set_tuning(self._h, C.byref(t))
        if rc != GG_OK:
            raise GGError(rc, "gg_index_set_tuning")

    def autotune(self, qbuf, qoff, prm: Params) -> dict:
        """gg_index_autotune on a sample batch; returns the kept choice."""
        q = _u8(qbuf)
        off = np.ascontiguousarray(qoff, dtype=np.int64)
        t = Tuning()
        rc = lib().gg_index_autotune(self._h, _ptr(q) if len(q) else None, _ptr(off),
                                     len(off) - 1, C.byref(prm), C.byref(t))
        if rc != GG_OK:
            raise GGError(rc, "gg_index_autotune")
        return {"grouping": GROUPINGS[t.grouping], "lane_steps": t.lane_steps,
                "wave_log2": t.wave_log2, "graph": t.graph, "graph_query_log2": t.graph_query_log2,
                "sample_ms": round(t.ms, 3)}

    def search(self, query, prm: Params, cap: int = 1024):
        """gg_search: returns (status, hits[:min(n, cap)], n)."""
        q = _u8(query)
        out = np.zeros(max(cap, 1), dtype=HIT_DTYPE)
        n = C.c_int32()
        rc = lib().gg_search(self._h, _ptr(q) if len(q) else None, len(q), C.byref(prm), _ptr(out),
                             cap, C.byref(n))
        if rc not in (GG_OK, GG_ETRUNC):
            return rc, np.zeros(0, HIT_DTYPE), 0
        return rc, out[: min(n.value, cap)].copy(), n.value

    def search_batch(self, qbuf, qoff, prm: Params, cap: int = 1024, stats: bool = False):
        """gg_search_batch: returns (status, list of hit arrays, counts, stats or None)."""
        b = _u8(qbuf)
        off = np.ascontiguousarray(qoff, dtype=np.int64)
        nq = len(off) - 1
        out = np.zeros(max(nq * cap, 1), dtype=HIT_DTYPE)
        nout = np.zeros(max(nq, 1), dtype=np.int32)
        st = np.zeros(max(nq, 1), dtype=STAT_DTYPE) if stats else None
        rc = lib().gg_search_batch(self._h, _ptr(b) if len(b) else None, _ptr(off), nq,
                                   C.byref(prm), _ptr(out), cap, _ptr(nout),
                                   _ptr(st) if stats else None)
        if rc not in (GG_OK, GG_ETRUNC):
            return rc, [], nout[:nq], None
        res = [out[i * cap: i * cap + min(int(nout[i]), cap)].copy() for i in range(nq)]
        return rc, res, nout[:nq].copy(), (st[:nq] if stats else None)

    def search_batch_into(self, qbuf: np.ndarray, qoff: np.ndarray, prm: Params, out: np.ndarray,
                          nout: np.ndarray, cap: int) -> int:
        """gg_search_batch into caller-owned arrays (out: n_q * cap hits, nout: n_q
        counts), with no per-query unpacking; returns the status."""
        nq = len(qoff) - 1
        assert qbuf.dtype == np.uint8 and qoff.dtype == np.int64 and out.dtype == HIT_DTYPE
        assert nout.dtype == np.int32 and len(out) >= nq * cap and len(nout) >= nq
        return lib().gg_search_batch(self._h, _ptr(qbuf) if len(qbuf) else None, _ptr(qoff), nq,
                                     C.byref(prm), _ptr(out), cap, _ptr(nout), None)

    def search_batch_device(self, dq: "DeviceBuffer", qoff, prm: Params, dout: "DeviceBuffer",
                            dn: "DeviceBuffer", cap: int, stats: bool = False):
        """gg_search_batch_device on device-resident queries and result buffers."""
        off = np.ascontiguousarray(qoff, dtype=np.int64)
        nq = len(off) - 1
        st = np.zeros(max(nq, 1), dtype=STAT_DTYPE) if stats else None
        rc = lib().gg_search_batch_device(self._h, dq.ptr, _ptr(off), nq, C.byref(prm), dout.ptr,
                                          cap, dn.ptr, _ptr(st) if stats else None)
        return rc, (st[:nq] if stats else None)

    # ---- per-stage GPU timing
    def profile(self, on: bool = True):
        rc = lib().gg_profile_enable(self._h, 1 if on else 0)
        if rc != GG_OK:
            raise GGError(rc, "gg_profile_enable")

    def profile_read(self, stage: str) -> dict:
        ms, la, un = C.c_double(), C.c_int64(), C.c_int64()
        rc = lib().gg_profile_read(self._h, stage.encode(), C.byref(ms), C.byref(la), C.byref(un))
        if rc != GG_OK:
            raise GGError(rc, "gg_profile_read")
        return {"ms": ms.value, "launches": la.value, "units": un.value}


class DeviceBuffer:
    """gg_device_alloc / gg_device_free: raw GPU memory for the device-resident form."""

    def __init__(self, nbytes: int, device: int = 0):
        p = C.c_void_p()
        rc = lib().gg_device_alloc(device, int(nbytes), C.byref(p))
        if rc != GG_OK:
            raise GGError(rc, "gg_device_alloc")
        self.ptr, self.nbytes, self.device = p, int(nbytes), device

    def upload(self, a: np.ndarray):
        a = np.ascontiguousarray(a)
        assert a.nbytes <= self.nbytes
        rc = lib().gg_memcpy_to_device(self.ptr, _ptr(a), a.nbytes)
        if rc != GG_OK:
            raise GGError(rc, "gg_memcpy_to_device")

    def download(self, a: np.ndarray) -> np.ndarray:
        assert a.flags.c_contiguous and a.nbytes <= self.nbytes
        rc = lib().gg_memcpy_to_host(_ptr(a), self.ptr, a.nbytes)
        if rc != GG_OK:
            raise GGError(rc, "gg_memcpy_to_host")
        return a

    def read_sum(self, nbytes: int) -> int:
        """gg_device_read: stream the first nbytes once on the GPU; their word sum."""
        v = C.c_uint64()
        rc = lib().gg_device_read(self.ptr, int(nbytes), C.byref(v))
        if rc != GG_OK:
            raise GGError(rc, "gg_device_read")
        return v.value

    def copy_from(self, other: "DeviceBuffer", nbytes: int):
        rc = lib().gg_device_copy(self.ptr, other.ptr, int(nbytes))
        if rc != GG_OK:
            raise GGError(rc, "gg_device_copy")

    def close(self):
        if getattr(self, "ptr", None) and self.ptr.value:
            lib().gg_device_free(self.device, self.ptr)
            self.ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """gg_server_create / gg_serve_submit / gg_serve_poll / gg_server_destroy."""

    def __init__(self, index: Index, prm: Params, hit_budget_bytes: int = 0, max_slots: int = 64):
        h = C.c_void_p()
        rc = lib().gg_server_create(index.handle, C.byref(prm), int(hit_budget_bytes), max_slots,
                                    C.byref(h))
        if rc != GG_OK:
            raise GGError(rc, "gg_server_create")
        self._h = h
        self._index = index  # keep the index alive while serving

    def submit(self, query) -> int:
        q = _u8(query)
        t = C.c_uint64()
        rc = lib().gg_serve_submit(self._h, _ptr(q) if len(q) else None, len(q), C.byref(t))
        if rc != GG_OK:
            raise GGError(rc, "gg_serve_submit")
        return t.value

    def poll(self, ticket: int, cap: int = 1024, timeout_us: int = 0):
        """Returns (status, hits, n); status GG_EAGAIN while pending."""
        out = np.zeros(max(cap, 1), dtype=HIT_DTYPE)
        n = C.c_int32()
        rc = lib().gg_serve_poll(self._h, ticket, _ptr(out), cap, C.byref(n), timeout_us)
        if rc in (GG_OK, GG_ETRUNC):
            return rc, out[: min(n.value, cap)].copy(), n.value
        return rc, np.zeros(0, HIT_DTYPE), 0

    def info(self) -> dict:
        """gg_server_info: admission totals and peaks."""
        t = ServerStats()
        rc = lib().gg_server_info(self._h, C.byref(t))
        if rc != GG_OK:
            raise GGError(rc, "gg_server_info")
        return {f: getattr(t, f) for f, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().gg_server_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
