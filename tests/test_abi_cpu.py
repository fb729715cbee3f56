"""The C-ABI library loads, exports every declared symbol and validates its
arguments before touching the GPU (runs without a GPU)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "fwht.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fwht_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_1607_01039_amd import _lib
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    from paper_1607_01039_amd import _lib
    decl = declared_symbols()
    assert len(decl) >= 10
    assert set(decl) == set(_lib.EXPORTS)
    for name in decl:
        assert hasattr(L, name), name


def test_version(L):
    assert L.fwht_version().startswith(b"fwht-gfx950")


def _buf():
    # 16-byte aligned host buffer; validation fails before it is ever used.
    b = (C.c_uint8 * 64)()
    base = C.addressof(b)
    return b, base + (-base % 16)


def test_int_validation(L):
    from paper_1607_01039_amd import _lib
    keep, p = _buf()
    assert L.fwht_int(None, 0, 4, None, None) == _lib.FWHT_E_INVAL
    assert L.fwht_int(C.c_void_p(p + 4), 0, 4, None, None) == _lib.FWHT_E_INVAL
    assert L.fwht_int(C.c_void_p(p), 7, 4, None, None) == _lib.FWHT_E_INVAL
    assert L.fwht_int(C.c_void_p(p), _lib.FWHT_I32, -1, None, None) == _lib.FWHT_E_RANGE
    assert L.fwht_int(C.c_void_p(p), _lib.FWHT_I32, 31, None, None) == _lib.FWHT_E_RANGE
    assert b"n <= 30" in L.fwht_last_error()
    th = _lib.fwht_thresh_t(5, 0.0, None, None, 4, None)
    assert L.fwht_int(C.c_void_p(p), _lib.FWHT_I32, 4, C.byref(th), None) == _lib.FWHT_E_INVAL
    th = _lib.fwht_thresh_t(5, 0.0, None, None, 4, p)
    assert L.fwht_int(C.c_void_p(p), _lib.FWHT_I32, 4, C.byref(th), None) == _lib.FWHT_E_INVAL


def test_float_validation(L):
    from paper_1607_01039_amd import _lib
    keep, p = _buf()
    assert L.fwht_float(None, 4, 1, 1, 0, None) == _lib.FWHT_E_INVAL
    assert L.fwht_float(C.c_void_p(p), 31, 1, 1, 0, None) == _lib.FWHT_E_RANGE
    assert L.fwht_float(C.c_void_p(p), 4, 0, 1, 0, None) == _lib.FWHT_E_INVAL
    assert L.fwht_float(C.c_void_p(p), 30, 1 << 12, 1, 0, None) == _lib.FWHT_E_RANGE
    assert L.fwht_float(C.c_void_p(p), 4, 1, 1, 9, None) == _lib.FWHT_E_INVAL
    # out of place: host-side checks only (nothing reaches a device)
    q = p + 64 * 4
    assert L.fwht_float_out(None, C.c_void_p(p), 4, 1, 1, 0, None) == _lib.FWHT_E_INVAL
    assert L.fwht_float_out(C.c_void_p(p), None, 4, 1, 1, 0, None) == _lib.FWHT_E_INVAL
    assert L.fwht_float_out(C.c_void_p(p), C.c_void_p(p + 4), 4, 1, 1, 0, None) == _lib.FWHT_E_INVAL  # misaligned
    assert L.fwht_float_out(C.c_void_p(p), C.c_void_p(p + 16), 4, 1, 1, 0, None) == _lib.FWHT_E_INVAL  # overlap
    assert L.fwht_float_out(C.c_void_p(p + 16), C.c_void_p(p), 4, 1, 1, 0, None) == _lib.FWHT_E_INVAL  # overlap
    assert b"overlap" in L.fwht_last_error()
    assert L.fwht_float_out(C.c_void_p(p), C.c_void_p(q), 31, 1, 1, 0, None) == _lib.FWHT_E_RANGE
    assert L.fwht_float_out(C.c_void_p(p), C.c_void_p(q), 4, 0, 1, 0, None) == _lib.FWHT_E_INVAL
    assert L.fwht_float_out(C.c_void_p(p), C.c_void_p(q), 4, 1, 1, 9, None) == _lib.FWHT_E_INVAL
    # matrix-core limits are checked before the copy is enqueued
    assert L.fwht_float_out(C.c_void_p(p), C.c_void_p(q), 3, 1, 1, 1, None) == _lib.FWHT_E_UNSUPPORTED
    assert L.fwht_float_out(C.c_void_p(p), C.c_void_p(p + (1 << 21)), 17, 1, 1, 2, None) == _lib.FWHT_E_UNSUPPORTED


def test_threshold_validation(L):
    from paper_1607_01039_amd import _lib
    keep, p = _buf()
    assert L.fwht_threshold(C.c_void_p(p), 0, 4, None, None) == _lib.FWHT_E_INVAL
    th = _lib.fwht_thresh_t(5, 0.0, p, p, 4, p)
    assert L.fwht_threshold(C.c_void_p(p), 9, 4, C.byref(th), None) == _lib.FWHT_E_INVAL
    assert L.fwht_threshold(C.c_void_p(p), 0, -2, C.byref(th), None) == _lib.FWHT_E_RANGE


def test_schedule_parsing(L):
    from paper_1607_01039_amd import _lib
    ok = [(0, 30, b"C14,S14c6,S14c6"), (0, 20, b"C12,S14c6:8"), (1, 25, b"C13,S13c5,S13c5:4"),
          (2, 16, b"C15:10,S12c5:6"), (0, 30, b"C16,S15c8:7,S15c8:7"), (2, 17, b"C16,S9c8:1"),
          (0, 30, b"C15pn,S15c8n:7,S16c8n:8"), (2, 20, b"C15p,S13c8:5"),
          (1, 30, b"C14pn,S14c5n:9,S13c6:5,S12c6:2"), (1, 34, b"C14pn,S14c7:7,S14c7:7,S13c7:6")]
    for dt, n, spec in ok:
        assert L.fwht_set_schedule(dt, n, spec) == 0, (spec, L.fwht_last_error())
        buf = C.create_string_buffer(128)
        assert L.fwht_get_schedule(dt, n, buf, 128) == 0 and buf.value == spec
        assert L.fwht_set_schedule(dt, n, None) == 0
    bad = [(0, 30, b"C14,S14c6"), (0, 20, b"S14c6,C14"), (0, 20, b"X9"), (0, 20, b"C14:0,S14c6"),
           (0, 20, b"C12:3,S14c6,S14c6"), (0, 16, b"C16"), (0, 20, b"C16:12,S12c8:8"), (2, 16, b"C16"), (0, 15, b"C15p"),
           (0, 20, b"C15p:12,S12c8:8"), (1, 20, b"C15p,S13c8:5"),
           # 8-byte entries: lane offsets of a row bit at stride 2^29 (2^32 bytes) no longer fit 32 bits
           (1, 30, b"C14pn,S14c5n:9,S13c6:6,S12c6:1"), (1, 32, b"C13,S13c5:8,S13c5:8,S13c5:3")]
    for dt, n, spec in bad:
        assert L.fwht_set_schedule(dt, n, spec) == _lib.FWHT_E_INVAL, spec


def test_default_schedules_cover_every_n(L):
    for dt, nmax in ((0, 30), (1, 35), (2, 30)):
        for n in range(1, nmax + 1):
            buf = C.create_string_buffer(128)
            assert L.fwht_get_schedule(dt, n, buf, 128) == 0
            assert L.fwht_set_schedule(dt, n, buf.value) == 0, (dt, n, buf.value, L.fwht_last_error())
            assert L.fwht_set_schedule(dt, n, None) == 0


def test_product_does_not_import_oracle():
    import subprocess, sys
    code = ("import sys, paper_1607_01039_amd as p; p._lib.lib();"
            "assert 'oracle' not in sys.modules, 'product imported the oracle'")
    subprocess.run([sys.executable, "-c", code], check=True, cwd=ROOT)


def test_fold_validation(L):
    from paper_1607_01039_amd import _lib
    import numpy as np
    keep, p = _buf()
    rows = np.array([0b0011, 0b0101, 0b1000], dtype=np.uint64)
    basis = np.zeros(4, dtype=np.uint64)
    rp, bp = rows.ctypes.data_as(C.c_void_p), basis.ctypes.data_as(C.c_void_p)
    x, u = C.c_void_p(p), C.c_void_p(p)
    assert L.fwht_fold(x, 7, 4, 3, rp, u, bp, None) == _lib.FWHT_E_INVAL
    assert L.fwht_fold(x, 0, 41, 3, rp, u, bp, None) == _lib.FWHT_E_RANGE
    assert L.fwht_fold(x, 0, 4, 5, rp, u, bp, None) == _lib.FWHT_E_RANGE
    assert L.fwht_fold(None, 0, 4, 3, rp, u, bp, None) == _lib.FWHT_E_INVAL
    assert L.fwht_fold(C.c_void_p(p + 4), 0, 4, 3, rp, u, bp, None) == _lib.FWHT_E_INVAL
    assert L.fwht_fold(x, 0, 4, 3, None, u, bp, None) == _lib.FWHT_E_INVAL
    assert L.fwht_fold(x, 0, 3, 3, rp, u, bp, None) == _lib.FWHT_E_INVAL  # row bit 3 >= n
    assert b"at or above" in L.fwht_last_error()
    dep = np.array([0b0011, 0b0101, 0b0110], dtype=np.uint64)  # third = first ^ second
    assert L.fwht_fold(x, 1, 4, 3, dep.ctypes.data_as(C.c_void_p), u, bp, None) == _lib.FWHT_E_INVAL
    assert b"dependent" in L.fwht_last_error()
    assert not basis.any()  # nothing written on failure
    assert L.fwht_fold_planted(0, 49, 3, rp, 0, 1, 2, u, bp, None) == _lib.FWHT_E_RANGE
    assert L.fwht_fold_planted(0, 4, 3, rp, 1 << 4, 1, 2, u, bp, None) == _lib.FWHT_E_INVAL
    assert L.fwht_fold_planted(0, 4, 3, rp, 0, 1, 2, None, bp, None) == _lib.FWHT_E_INVAL
    assert L.fwht_subspace_hits(x, 4, None, 3, bp, None) == _lib.FWHT_E_INVAL
    assert L.fwht_subspace_hits(x, 4, x, 37, bp, None) == _lib.FWHT_E_RANGE
    assert L.fwht_subspace_hits(x, 4, x, 3, None, None) == _lib.FWHT_E_INVAL
    assert L.fwht_subspace_hits(x, 0, x, 3, bp, None) == _lib.FWHT_OK  # nothing to map


def test_prime_omega_validation(L):
    from paper_1607_01039_amd import _lib
    keep, p = _buf()
    assert L.fwht_prime_omega(None, 1, 10, None) == _lib.FWHT_E_INVAL
    assert L.fwht_prime_omega(C.c_void_p(p + 4), 1, 10, None) == _lib.FWHT_E_INVAL
    assert L.fwht_prime_omega(C.c_void_p(p), 2, 10, None) == _lib.FWHT_E_INVAL
    assert L.fwht_prime_omega(C.c_void_p(p), 1, 33, None) == _lib.FWHT_E_RANGE
    assert L.fwht_prime_omega(C.c_void_p(p), 1, -1, None) == _lib.FWHT_E_RANGE


def test_missing_library_fails_loudly():
    # With the HIP library absent the binding raises; there is no CPU fallback.
    import subprocess, sys
    code = ("import paper_1607_01039_amd._lib as L\n"
            "L.LIB_PATH = '/nonexistent/libfwht.so'\n"
            "L._lib = None\n"
            "try:\n"
            "    L.lib()\n"
            "except ImportError as e:\n"
            "    assert 'missing' in str(e)\n"
            "else:\n"
            "    raise SystemExit('no error')\n")
    subprocess.run([sys.executable, "-c", code], check=True, cwd=ROOT)


def test_batched_validation(L):
    # log2n must lie in [2, 16] as the header states; offsets multiples of 4.
    from paper_1607_01039_amd import _lib
    import numpy as np
    keep, p = _buf()
    x = C.c_void_p(p)
    off = np.array([0, 64], dtype=np.int64)

    def call(lg, offs=off, count=2, prec=0, data=x):
        lg = np.asarray(lg, dtype=np.int32)
        return L.fwht_batched(data, offs.ctypes.data_as(C.c_void_p), lg.ctypes.data_as(C.c_void_p), count, 1,
                              prec, None)

    for bad in (0, 1, 17, -3):
        assert call([4, bad]) == _lib.FWHT_E_RANGE, bad
        assert b"[2, 16]" in L.fwht_last_error()
    assert call([4, 4], offs=np.array([0, 66], dtype=np.int64)) == _lib.FWHT_E_INVAL
    assert call([4, 4], count=0) == _lib.FWHT_E_INVAL
    assert call([4, 4], prec=7) == _lib.FWHT_E_INVAL
    assert call([4, 4], data=C.c_void_p(p + 4)) == _lib.FWHT_E_INVAL
    assert call([4, 4], data=None) == _lib.FWHT_E_INVAL


def test_batched_noalloc_validation(L):
    # The allocation-free variant validates like fwht_batched and refuses more
    # transforms than its fixed work-list array holds.
    from paper_1607_01039_amd import _lib
    import numpy as np
    keep, p = _buf()
    x = C.c_void_p(p)
    big = _lib.FWHT_NOALLOC_MAX_TRANSFORMS + 1
    off = (np.arange(big, dtype=np.int64) * 4)
    lg = np.full(big, 2, dtype=np.int32)
    args = (off.ctypes.data_as(C.c_void_p), lg.ctypes.data_as(C.c_void_p))
    assert L.fwht_batched_noalloc(x, *args, big, 1, 0, None) == _lib.FWHT_E_RANGE
    assert b"limit" in L.fwht_last_error()
    lg[1] = 17
    assert L.fwht_batched_noalloc(x, *args, 2, 1, 0, None) == _lib.FWHT_E_RANGE
    lg[1] = 2
    off[1] = 6
    assert L.fwht_batched_noalloc(x, *args, 2, 1, 0, None) == _lib.FWHT_E_INVAL
    assert L.fwht_batched_noalloc(x, *args, 0, 1, 0, None) == _lib.FWHT_E_INVAL
    assert L.fwht_batched_noalloc(x, *args, 1, 1, 5, None) == _lib.FWHT_E_INVAL
    assert L.fwht_batched_noalloc(None, *args, 1, 1, 0, None) == _lib.FWHT_E_INVAL


def test_batched_tile_groups_parsing(L):
    from paper_1607_01039_amd import _lib
    buf = C.create_string_buffer(64)
    for spec in (b"16:2-16", b"16:16,15:2-15", b"16:16,15:15,14:2-14", b"15:2-15,16:16"):
        assert L.fwht_set_batched_tiles(0, spec) == 0, (spec, L.fwht_last_error())
        assert L.fwht_get_batched_tiles(0, buf, 64) == 0 and buf.value == spec
    assert L.fwht_set_batched_tiles(1, b"16:2-16") == 0
    bad = [(0, b"16:2-15"), (0, b"16:2-16,15:15"), (0, b"17:2-16"), (0, b"13:2-13,16:14-16"), (0, b"15:2-16"),
           (0, b"16:1-16"), (0, b"16:x"), (1, b"16:16,15:2-15"), (0, b"16:16,15:15,14:3-14,14:2"), (5, b"16:2-16")]
    for prec, spec in bad:
        assert L.fwht_set_batched_tiles(prec, spec) == _lib.FWHT_E_INVAL, spec
    assert L.fwht_set_batched_tiles(0, None) == 0 and L.fwht_set_batched_tiles(1, None) == 0
    small = C.create_string_buffer(3)
    assert L.fwht_get_batched_tiles(0, small, 3) == _lib.FWHT_E_CAPACITY


def test_batched_launch_mode_switch(L):
    """Direct launches by default; the graph-replay setting reads back and restores."""
    assert L.fwht_get_batched_graphs() == 0
    assert L.fwht_set_batched_graphs(1) == 0 and L.fwht_get_batched_graphs() == 1
    assert L.fwht_set_batched_graphs(7) == 0 and L.fwht_get_batched_graphs() == 1
    assert L.fwht_set_batched_graphs(0) == 0 and L.fwht_get_batched_graphs() == 0


def test_norms_validation(L):
    """Argument checks of fwht_norms that come before any device call."""
    from paper_1607_01039_amd import _lib
    keep, p = _buf()
    off = (C.c_int64 * 1)(0)
    lg = (C.c_int32 * 1)(4)
    v = C.c_void_p(p)
    for args in ((None, v, None, off, lg, 1, v), (v, None, None, off, lg, 1, v), (v, v, None, None, lg, 1, v),
                 (v, v, None, off, None, 1, v), (v, v, None, off, lg, 1, None)):
        assert L.fwht_norms(*args, None) == _lib.FWHT_E_INVAL
    assert b"NULL" in L.fwht_last_error()
    assert L.fwht_norms(v, v, None, off, lg, 0, v, None) == _lib.FWHT_E_INVAL
    assert L.fwht_norms(v, v, None, off, lg, (1 << 23) + 1, v, None) == _lib.FWHT_E_RANGE


def test_autotuner_candidates_parse(L):
    """Every schedule the autotuner would time names compiled variants at
    heights the library accepts, including the held (two workgroups per CU)
    strided tiles; the held and wide strided variants it knows are exactly
    the compiled ones."""
    import paper_1607_01039_amd as F
    from paper_1607_01039_amd import autotune as A
    codes = {"int32": 0, "int64": 1, "float32": 2}
    for dt, code in codes.items():
        names = set(F.list_variants(dt))
        held = {v for v in names if v.startswith("S") and v.rstrip("n").endswith("p")}
        assert {v for v in A.HELD.get(dt, {}).values()} | {v + "n" for v in A.HELD.get(dt, {}).values()} == held
        wide = {v for v in names if v.rstrip("n").endswith("w")}
        assert {v for v in A.WIDE.get(dt, {}).values()} | {v + "n" for v in A.WIDE.get(dt, {}).values()} == wide
        for n in (20, 24, 28, 30):
            cands = A.candidates(dt, n)
            assert cands
            for spec in cands:
                for part in spec.split(","):
                    assert part.split(":")[0] in names, (dt, n, spec)
                rc = L.fwht_set_schedule(code, n, spec.encode())
                assert rc == 0, (dt, n, spec, L.fwht_last_error())
            assert L.fwht_set_schedule(code, n, None) == 0
