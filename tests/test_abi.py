"""C-ABI checks that need no GPU: the library loads, exports every function
include/xdrop.h declares, packs reads in the documented layout and rejects bad
arguments before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2001_10049_amd as xd
from paper_2001_10049_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(xd_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = declared_functions()
    assert names, "no declarations found"
    assert names == set(_lib.EXPORTS)
    for name in names:
        assert hasattr(lib, name), name


def test_pack_layout():
    rng = np.random.default_rng(0)
    lens = [0, 1, 15, 16, 17, 300, 1000]
    reads = [rng.integers(0, 4, L, dtype=np.uint8) for L in lens]
    length = np.array(lens, np.uint32)
    off = np.concatenate([[0], np.cumsum(length)[:-1]]).astype(np.uint64)
    codes = np.concatenate(reads)
    words, woff = xd.pack_reads(codes, off, length)
    for r, seq in enumerate(reads):
        assert woff[r] % 16 == 0  # 64-byte aligned reads
        for u, c in enumerate(seq):
            w = int(words[int(woff[r]) + u // 16])
            assert (w >> (2 * (u % 16))) & 3 == c
        # zero padding after the last base
        nw = (len(seq) + 15) // 16
        if len(seq) % 16:
            tail = int(words[int(woff[r]) + nw - 1]) >> (2 * (len(seq) % 16))
            assert tail == 0
    assert len(words) == int(woff[-1]) + ((1000 + 15) // 16 + 15) // 16 * 16


def test_pack_rejects_bad_codes():
    codes = np.array([0, 1, 4], np.uint8)
    with pytest.raises(xd.XdropError):
        xd.pack_reads(codes, np.array([0], np.uint64), np.array([3], np.uint32))


def test_align_batch_argument_errors_without_device():
    lib = _lib.load()
    fake = ctypes.c_void_p(0)
    args = [None, None, None, 0, 1, 17, 1, -1, -1, None, None, None, None, None, None]
    # null store
    assert lib.xd_align_batch(fake, *args) == _lib.XD_EINVAL
    assert b"store" in lib.xd_last_error()


@pytest.mark.parametrize("k,m,mm,g", [(0, 1, -1, -1), (17, 0, -1, -1), (17, 1, 1, -1),
                                      (17, 1, -1, 0), (17, 1001, -1, -1), (17, 1, -1, -1001),
                                      (17, 1, -1001, -1), (17, 5, 5, -1)])
def test_align_batch_rejects_bad_scoring(k, m, mm, g):
    lib = _lib.load()
    dummy = ctypes.c_void_p(1)  # never dereferenced: scalar checks come first
    rc = lib.xd_align_batch(dummy, None, None, None, 5, 1, k, m, mm, g, None, None, None,
                            None, None, None)
    assert rc == _lib.XD_EINVAL


def test_align_batch_rejects_bad_scalar_x():
    lib = _lib.load()
    dummy = ctypes.c_void_p(1)
    for x in (-1, _lib.X_MAX + 1):
        rc = lib.xd_align_batch(dummy, None, None, None, x, 1, 17, 1, -1, -1, None, None,
                                None, None, None, None)
        assert rc == _lib.XD_EINVAL


def test_store_create_rejects_bad_layout():
    lib = _lib.load()
    h = ctypes.c_void_p()
    words = np.zeros(4, np.uint32)
    woff = np.array([0], np.uint64)
    length = np.array([100], np.uint32)  # needs 7 words, only 4 given
    rc = lib.xd_store_create(words.ctypes.data_as(ctypes.c_void_p), 4,
                             woff.ctypes.data_as(ctypes.c_void_p),
                             length.ctypes.data_as(ctypes.c_void_p), 1, ctypes.byref(h))
    assert rc == _lib.XD_EINVAL
    length = np.array([_lib.READ_MAX + 1], np.uint32)
    rc = lib.xd_store_create(words.ctypes.data_as(ctypes.c_void_p), 4,
                             woff.ctypes.data_as(ctypes.c_void_p),
                             length.ctypes.data_as(ctypes.c_void_p), 1, ctypes.byref(h))
    assert rc == _lib.XD_EINVAL


def test_find_overlaps_rejects_null_store():
    lib = _lib.load()
    cnt = _lib.OverlapCounts()
    rc = lib.xd_find_overlaps(ctypes.c_void_p(0), 17, 8, 0, 0, 0, None, None, 0, None,
                              ctypes.byref(cnt), None)
    assert rc == _lib.XD_EINVAL and b"store" in lib.xd_last_error()


def test_find_overlaps_strands_rejects_bad_strand():
    lib = _lib.load()
    cnt = _lib.OverlapCounts()
    for strands in (0, 3, -1):
        # the dummy store is never dereferenced: the strand is checked first
        rc = lib.xd_find_overlaps_strands(ctypes.c_void_p(1), 17, 8, 0, 0, strands, 0, None,
                                          None, None, 0, None, ctypes.byref(cnt), None)
        assert rc == _lib.XD_EINVAL and b"strands" in lib.xd_last_error()


def test_banded_traceback_argument_errors_without_device():
    lib = _lib.load()
    dummy = ctypes.c_void_p(1)  # never dereferenced: scalar checks come first

    def call(store, w_scalar=32, n=1, k=17, m=1, mm=-1, g=-1, arrays=None):
        a = arrays or [None] * 8
        return lib.xd_banded_traceback(store, None, None, None, w_scalar, n, k, m, mm, g, 64, 0,
                                       *a, None)

    assert call(ctypes.c_void_p(0)) == _lib.XD_EINVAL
    assert b"store" in lib.xd_last_error()
    assert call(dummy, k=0) == _lib.XD_EINVAL
    assert call(dummy, mm=2) == _lib.XD_EINVAL
    # banded scoring stays within +-127
    assert call(dummy, m=128) == _lib.XD_EINVAL and b"127" in lib.xd_last_error()
    assert call(dummy, g=-128) == _lib.XD_EINVAL
    assert call(dummy, mm=-128) == _lib.XD_EINVAL
    assert call(dummy, w_scalar=_lib.BAND_MAX + 1) == _lib.XD_EINVAL
    assert call(dummy, w_scalar=-1) == _lib.XD_EINVAL
    assert call(dummy, n=1) == _lib.XD_EINVAL          # null task and result arrays
    assert call(dummy, n=(1 << 30) + 1) == _lib.XD_EINVAL
    assert call(dummy, n=0) == _lib.XD_OK              # nothing to do


def _al(b):
    return (b + 255) // 256 * 256


def test_batch_scratch_bytes_layout():
    # per task two 24-byte extension results and six 4-byte lists per
    # extension, each array rounded up to 256 bytes, 4,352 fixed bytes, and
    # the resume states of the 64-, 128-, 256- and 512-cell windows (64 << t
    # rows, t = 0..3): 2n / (8, 16, 32, 256) states of 64 + 8 * rows bytes,
    # each pool rounded up to 256 bytes
    lib = _lib.load()
    for n in (0, 1, 2, 5, 31, 32, 33, 1000, 12345, 10**6):
        want = _al(48 * n) + 6 * _al(8 * n) + 4352
        for t, div in ((0, 8), (1, 16), (2, 32), (3, 256)):
            want += _al(-(-2 * n // div) * (64 + 8 * (64 << t)))
        assert lib.xd_batch_scratch_bytes(None, n, None) == want, n
    bad = _lib.Tuning(3, 0, 0, 0, 0, 0)  # waves_per_cu must be a multiple of 4
    assert lib.xd_batch_scratch_bytes(ctypes.c_void_p(1), 10, ctypes.byref(bad)) == 0


def test_server_request_bytes_cover_the_batch():
    # a request is charged at least its in/out buffer plus the whole batch
    # scratch of a batch of its size; several requests packed together are
    # charged at least what their batch takes
    lib = _lib.load()
    for n in range(1, 10001):
        need = 52 * n + lib.xd_batch_scratch_bytes(None, n, None)
        assert lib.xd_server_request_bytes(n) >= need, n
    sizes = [1, 7, 300, 1000, 4096, 9999]
    packed = sum(sizes)
    assert sum(lib.xd_server_request_bytes(s) for s in sizes) >= (
        _al(52 * packed) + lib.xd_batch_scratch_bytes(None, packed, None))


def test_server_create_rejects_bad_scoring():
    lib = _lib.load()
    h = ctypes.c_void_p()
    for k, m, mm, g in [(0, 1, -1, -1), (17, 0, -1, -1), (17, 1, 1, -1), (17, 1, -1, 0),
                        (17, 1001, -1, -1), (17, 1, -1, -1001)]:
        cfg = _lib.ServerConfig(1 << 30, 1, 0, 0, k, m, mm, g, _lib.Tuning())
        # the dummy store is never dereferenced: the scheme is checked first
        rc = lib.xd_server_create(ctypes.c_void_p(1), ctypes.byref(cfg), ctypes.byref(h))
        assert rc == _lib.XD_EINVAL and not h.value, (k, m, mm, g)
        msg = lib.xd_last_error()
        assert b"k must" in msg or b"match" in msg or b"mismatch" in msg or b"gap" in msg
