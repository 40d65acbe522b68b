"""The index file format, checked on the host: a file written here from the
documented layout loads as far as the device step (no GPU is needed to reach it),
and damaged variants are refused with GG_EIO or GG_EINVAL before any device use.
"""
import struct

import numpy as np
import pytest

from paper_1507_02987_amd import gg

M64 = (1 << 64) - 1


def file_hash(body: bytes) -> int:
    """The layout's check: 64-bit little-endian words, last one zero-padded; each is
    xored in, then multiplied by 0xff51afd7ed558ccd and xored with itself >> 33."""
    body = body + b"\0" * (-len(body) % 8)
    h = 0x9E3779B97F4A7C15
    for (w,) in struct.iter_unpack("<Q", body):
        h ^= w
        h = (h * 0xFF51AFD7ED558CCD) & M64
        h ^= h >> 33
    return h


def tiny_index_file(k=1, seqs=(b"ACGTAC", b"GGT")):
    """A plain k = 1 index of two sequences, built by hand."""
    codes = {"A": 0, "C": 1, "G": 2, "T": 3}
    starts = np.cumsum([0] + [len(s) for s in seqs]).astype(np.int64)
    lists = {c: [] for c in range(4 ** k)}
    for si, sq in enumerate(seqs):
        for pos in range(0, len(sq) - k + 1, k):
            c = 0
            for ch in sq[pos:pos + k].decode():
                c = c * 4 + codes[ch]
            lists[c].append((si, pos))
    heads = np.cumsum([0] + [len(lists[c]) for c in range(4 ** k)]).astype(np.uint32)
    post = np.array([p for c in range(4 ** k) for p in lists[c]], np.int32).reshape(-1, 2)
    bases = b"".join(seqs).decode()
    n_bases = len(bases)
    n_words = (n_bases + 15) // 16 + 1
    bank = np.zeros(n_words, np.uint32)
    for i, ch in enumerate(bases):
        bank[i // 16] |= codes[ch] << (30 - 2 * (i % 16))
    hdr = struct.pack("<I3iII5q", 1, k, k, 1, (1 << k) - 1, 0, len(seqs), n_bases, len(post),
                      max(len(s) for s in seqs), n_words)
    body = hdr + starts.tobytes() + heads.tobytes() + post.tobytes() + bank.tobytes()
    return b"GGINDEX1" + body + struct.pack("<Q", file_hash(body))


def load_status(path):
    h = gg.C.c_void_p()
    rc = gg.lib().gg_index_load(str(path).encode(), 0, gg.C.byref(h))
    if rc == gg.GG_OK:
        gg.lib().gg_index_free(h)
    return rc


def test_layout_hand_written_file_passes_every_check(tmp_path):
    p = tmp_path / "ok.ggi"
    p.write_bytes(tiny_index_file())
    # with no GPU the load stops at the device; on a GPU it succeeds
    assert load_status(p) in (gg.GG_OK, gg.GG_EDEVICE)


@pytest.mark.parametrize("damage", ["magic", "truncate", "extend", "flip_bank", "hash"])
def test_damaged_files_are_refused(tmp_path, damage):
    b = bytearray(tiny_index_file())
    if damage == "magic":
        b[0:8] = b"GGINDEX2"
    elif damage == "truncate":
        b = b[:-3]
    elif damage == "extend":
        b += b"\0"
    elif damage == "flip_bank":
        b[-12] ^= 0x40
    elif damage == "hash":
        b[-1] ^= 1
    p = tmp_path / f"{damage}.ggi"
    p.write_bytes(bytes(b))
    assert load_status(p) == gg.GG_EIO


def rehash(b: bytearray) -> bytes:
    body = bytes(b[8:-8])
    return bytes(b[:-8]) + struct.pack("<Q", file_hash(body))


@pytest.mark.parametrize("field,value", [("k", 0), ("span", 40), ("strands", 3), ("mask", 3),
                                         ("n_words", 9)])
def test_inconsistent_headers_are_refused(tmp_path, field, value):
    b = bytearray(tiny_index_file())
    at = {"k": 12, "span": 16, "strands": 20, "mask": 24, "n_words": 64}[field]
    fmt = "<q" if field == "n_words" else "<i"
    struct.pack_into(fmt, b, at, value)
    p = tmp_path / f"{field}.ggi"
    p.write_bytes(rehash(b))
    assert load_status(p) in (gg.GG_EINVAL, gg.GG_EIO)


def test_out_of_range_posting_is_refused(tmp_path):
    b = bytearray(tiny_index_file())
    n_seqs = 2
    at = 72 + 8 * (n_seqs + 1) + 4 * (4 + 1)  # first posting
    struct.pack_into("<ii", b, at, 0, 6)  # a window past the end of sequence 0 (6 bases)
    p = tmp_path / "post.ggi"
    p.write_bytes(rehash(b))
    assert load_status(p) == gg.GG_EINVAL
    struct.pack_into("<ii", b, at, 5, 0)  # no sequence 5
    p.write_bytes(rehash(b))
    assert load_status(p) == gg.GG_EINVAL


def test_missing_file(tmp_path):
    assert load_status(tmp_path / "none.ggi") == gg.GG_EIO
