"""CPU oracle for the Walsh-Hadamard transform and its threshold pass.

TEST INFRASTRUCTURE.  Only the test-suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product (the
HIP library and its Python binding) never imports it, and it imports nothing
from the product.

The arithmetic lives in ``wht_oracle.c`` (plain C, built with gcc into
``liboracle.so`` by ``build()``); this module only marshals numpy arrays.

Functions follow section 2 (Eq. 2: y_i = sum_j (-1)^<i,j> x_j, natural order,
unnormalised) and the algorithms of Fig. 1 (serial in-place butterflies),
Fig. 2 (fork-join parallel decomposition) and Fig. 3 (external block scheme).
Section 5.1's linear space reduction (the fold u_j = sum_{A i = j} x_i and
the index map k' -> A^T k') is here too, with a plain GF(2) elimination
(canonical basis, preimage of one reduced index) in Python, and the prime-factor
counts Omega(i) of the workload announced in section 4.3.
Integer results are wrap-around (mod 2^32 for int32 data, mod 2^64 for int64);
floating point is IEEE double on the exactly up-cast input.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "wht_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


def build(out: str = LIB, mutant: int = 0) -> str:
    """Compile the oracle with gcc (optionally with a planted mistake)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
           f"-DORACLE_MUTANT={int(mutant)}", "-o", out, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return out


class Oracle:
    """ctypes view of one build of ``wht_oracle.c``."""

    def __init__(self, path: str = LIB):
        if not os.path.exists(path):
            build(path)
        L = C.CDLL(path)
        self._L = L
        L.oracle_mutant.restype = C.c_int
        self.mutant = L.oracle_mutant()
        L.wht_def_at_u64.argtypes = [_u64p, C.c_int, C.c_uint64]
        L.wht_def_at_u64.restype = C.c_uint64
        L.wht_def_u64.argtypes = [_u64p, C.c_int, _u64p]
        L.wht_def_at_i32.argtypes = [_i32p, C.c_int, C.c_uint64]
        L.wht_def_at_i32.restype = C.c_int64
        L.wht_def_at_i64.argtypes = [_i64p, C.c_int, C.c_uint64]
        L.wht_def_at_i64.restype = C.c_uint64
        L.wht_def_at_f64.argtypes = [_f64p, C.c_int, C.c_uint64]
        L.wht_def_at_f64.restype = C.c_double
        L.wht_def_f64.argtypes = [_f64p, C.c_int, _f64p]
        L.wht_fig1_u32.argtypes = [_u32p, C.c_int]
        L.wht_fig1_u64.argtypes = [_u64p, C.c_int]
        L.wht_fig1_f64.argtypes = [_f64p, C.c_int]
        L.wht_fig2_u32.argtypes = [_u32p, C.c_int, C.c_int]
        L.wht_fig2_u32.restype = C.c_int
        L.wht_fig2_u64.argtypes = [_u64p, C.c_int, C.c_int]
        L.wht_fig2_u64.restype = C.c_int
        L.wht_fig3_u64.argtypes = [_u64p, C.c_int, C.c_int]
        L.wht_fig3_u64.restype = C.c_int
        L.threshold_i32.argtypes = [_i32p, C.c_uint64, C.c_int64, _u64p, _i32p, C.c_uint64]
        L.threshold_i32.restype = C.c_uint64
        L.threshold_i64.argtypes = [_i64p, C.c_uint64, C.c_int64, _u64p, _i64p, C.c_uint64]
        L.threshold_i64.restype = C.c_uint64
        L.threshold_f64.argtypes = [_f64p, C.c_uint64, C.c_double, _u64p, _f64p, C.c_uint64]
        L.threshold_f64.restype = C.c_uint64
        L.wht_orthonormal_scale.argtypes = [C.c_int]
        L.wht_orthonormal_scale.restype = C.c_double
        L.wht_batch_f64.argtypes = [_f64p, C.c_int, C.c_uint64, C.c_int]
        L.wht_ragged_f64.argtypes = [_f64p, _i64p, _i32p, C.c_uint64, C.c_int]
        L.norms_f64.argtypes = [_f32p, _f32p, C.c_void_p, _i64p, _i32p, C.c_uint64,
                                _f64p, _f64p, _f64p]
        L.fold_u64.argtypes = [_u64p, C.c_int, _u64p, C.c_int, _u64p]
        L.fold_u32.argtypes = [_u32p, C.c_int, _u64p, C.c_int, _u32p]
        L.subspace_index.argtypes = [_u64p, C.c_int, C.c_uint64]
        L.subspace_index.restype = C.c_uint64
        L.prime_omega.argtypes = [C.c_uint64, _i32p, C.c_int]
        L.prime_omega.restype = C.c_int
        L.kf_sum.argtypes = [C.c_void_p, C.c_int, C.c_uint64, C.c_uint64, C.c_int, _u64p, C.c_int, C.c_int]
        L.kf_sum.restype = C.c_uint64
        L.sumsq_mod.argtypes = [C.c_void_p, C.c_int, C.c_uint64, C.c_int, C.c_int]
        L.sumsq_mod.restype = C.c_uint64
        L.prime_omega_at.argtypes = [C.c_uint64]
        L.prime_omega_at.restype = C.c_int32

    # ---- Eq. 2 written out ------------------------------------------------
    def wht_def(self, x: np.ndarray) -> np.ndarray:
        """Eq. 2 by definition, O(4^n).  int -> mod 2^64 (as int64), float -> f64."""
        n = _log2(x.size)
        if np.issubdtype(x.dtype, np.floating):
            xin = np.ascontiguousarray(x, dtype=np.float64)
            y = np.empty_like(xin)
            self._L.wht_def_f64(xin, n, y)
            return y
        xin = np.ascontiguousarray(x.astype(np.int64)).view(np.uint64)
        y = np.empty_like(xin)
        self._L.wht_def_u64(xin, n, y)
        return y.view(np.int64)

    def wht_def_at(self, x: np.ndarray, ks) -> np.ndarray:
        """Selected coefficients y_k by definition, O(2^n) each."""
        n = _log2(x.size)
        ks = [int(k) for k in ks]
        if x.dtype == np.int32:
            return np.array([self._L.wht_def_at_i32(x, n, k) for k in ks], dtype=np.int64)
        if x.dtype == np.int64:
            return np.array([self._L.wht_def_at_i64(x, n, k) for k in ks],
                            dtype=np.uint64).view(np.int64)
        xin = np.ascontiguousarray(x, dtype=np.float64)
        return np.array([self._L.wht_def_at_f64(xin, n, k) for k in ks], dtype=np.float64)

    # ---- Fig. 1 -------------------------------------------------------------
    def wht_fig1(self, x: np.ndarray) -> np.ndarray:
        """Fig. 1 on a copy.  int32 -> wrap mod 2^32, int64 -> mod 2^64, float -> f64."""
        n = _log2(x.size)
        if x.dtype == np.int32:
            b = np.array(x, dtype=np.int32, copy=True).view(np.uint32)
            self._L.wht_fig1_u32(b, n)
            return b.view(np.int32)
        if x.dtype == np.int64:
            b = np.array(x, dtype=np.int64, copy=True).view(np.uint64)
            self._L.wht_fig1_u64(b, n)
            return b.view(np.int64)
        b = np.array(x, dtype=np.float64, copy=True)
        self._L.wht_fig1_f64(b, n)
        return b

    def wht_fig1_inplace(self, x: np.ndarray) -> None:
        """Fig. 1 in place on an int32/int64/float64 array."""
        n = _log2(x.size)
        if x.dtype == np.int32:
            self._L.wht_fig1_u32(x.view(np.uint32), n)
        elif x.dtype == np.int64:
            self._L.wht_fig1_u64(x.view(np.uint64), n)
        elif x.dtype == np.float64:
            self._L.wht_fig1_f64(x, n)
        else:
            raise TypeError(x.dtype)

    # ---- Fig. 2 / Fig. 3 ---------------------------------------------------
    def wht_fig2_inplace(self, x: np.ndarray, q: int) -> None:
        """Fig. 2 with m = 2^q threads, in place (int32 or int64)."""
        n = _log2(x.size)
        if x.dtype == np.int32:
            rc = self._L.wht_fig2_u32(x.view(np.uint32), n, q)
        elif x.dtype == np.int64:
            rc = self._L.wht_fig2_u64(x.view(np.uint64), n, q)
        else:
            raise TypeError(x.dtype)
        if rc != 0:
            raise ValueError(f"fig2: q={q} invalid for n={n}")

    def wht_fig2(self, x: np.ndarray, q: int) -> np.ndarray:
        b = np.array(x, copy=True)
        self.wht_fig2_inplace(b, q)
        return b

    def wht_fig3(self, x: np.ndarray, B: int) -> np.ndarray:
        """Fig. 3 with in-memory capacity 2^B on a copy (int64)."""
        n = _log2(x.size)
        b = np.array(x, dtype=np.int64, copy=True).view(np.uint64)
        if self._L.wht_fig3_u64(b, n, B) != 0:
            raise ValueError("fig3: bad B")
        return b.view(np.int64)

    # ---- threshold pass -----------------------------------------------------
    def threshold(self, y: np.ndarray, T, cap: int | None = None):
        """All (k, y_k) with |y_k| > T in ascending k.  Returns (idx, val, count)."""
        y = np.ascontiguousarray(y)
        if cap is None:
            cap = y.size
        idx = np.zeros(max(cap, 1), dtype=np.uint64)
        if y.dtype == np.int32:
            val = np.zeros(max(cap, 1), dtype=np.int32)
            cnt = self._L.threshold_i32(y, y.size, int(T), idx, val, cap)
        elif y.dtype == np.int64:
            val = np.zeros(max(cap, 1), dtype=np.int64)
            cnt = self._L.threshold_i64(y, y.size, int(T), idx, val, cap)
        else:
            yd = np.ascontiguousarray(y, dtype=np.float64)
            val = np.zeros(max(cap, 1), dtype=np.float64)
            cnt = self._L.threshold_f64(yd, yd.size, float(T), idx, val, cap)
        k = min(cnt, cap)
        return idx[:k], val[:k], int(cnt)

    # ---- float transforms ---------------------------------------------------
    def orthonormal_scale(self, n: int) -> float:
        return self._L.wht_orthonormal_scale(n)

    def wht_batch(self, x: np.ndarray, n: int, normalize: bool) -> np.ndarray:
        """Rows of 2^n entries (any leading shape), each transformed in f64."""
        b = np.array(x, dtype=np.float64, copy=True).reshape(-1)
        batch = b.size >> n
        assert batch << n == b.size
        self._L.wht_batch_f64(b, n, batch, int(bool(normalize)))
        return b.reshape(x.shape)

    def wht_ragged(self, x: np.ndarray, off: np.ndarray, lg: np.ndarray,
                   normalize: bool) -> np.ndarray:
        b = np.array(x, dtype=np.float64, copy=True)
        self._L.wht_ragged_f64(b, np.ascontiguousarray(off, dtype=np.int64),
                               np.ascontiguousarray(lg, dtype=np.int32),
                               len(off), int(bool(normalize)))
        return b

    def norms(self, x: np.ndarray, y: np.ndarray, r, off: np.ndarray, lg: np.ndarray):
        """Per-transform (sum x^2, sum y^2, sum (y - r)^2) in double."""
        cnt = len(off)
        sx = np.zeros(cnt); sy = np.zeros(cnt); se = np.zeros(cnt)
        rp = None
        if r is not None:
            r = np.ascontiguousarray(r, dtype=np.float64)
            rp = r.ctypes.data_as(C.c_void_p)
        self._L.norms_f64(np.ascontiguousarray(x, dtype=np.float32),
                          np.ascontiguousarray(y, dtype=np.float32), rp,
                          np.ascontiguousarray(off, dtype=np.int64),
                          np.ascontiguousarray(lg, dtype=np.int32), cnt, sx, sy, se)
        return sx, sy, se

    def grad_weighted_square(self, x: np.ndarray, w: np.ndarray, n: int) -> np.ndarray:
        """Gradient of L = sum_{b,k} w_bk (Y x_b)_k^2 with Y the orthonormal WHT.

        Y is symmetric and orthogonal, so dL/dx_b = 2 Y (w_b * Y x_b) (in f64).
        """
        y = self.wht_batch(x, n, True)
        return self.wht_batch(2.0 * np.asarray(w, dtype=np.float64) * y, n, True)

    # ---- section 5.1: linear space reduction --------------------------------
    def fold(self, x: np.ndarray, rows, m: int) -> np.ndarray:
        """u_j = sum_{i : A i = j} x_i for the map A with the given m rows
        (bit t of A i is the parity of rows[t] & i); int32 or int64, wrapping."""
        n = _log2(x.size)
        r = np.ascontiguousarray(np.asarray(rows, dtype=np.uint64))
        assert r.size == m
        if x.dtype == np.int32:
            u = np.empty(1 << m, dtype=np.uint32)
            self._L.fold_u32(np.ascontiguousarray(x).view(np.uint32), n, r, m, u)
            return u.view(np.int32)
        if x.dtype == np.int64:
            u = np.empty(1 << m, dtype=np.uint64)
            self._L.fold_u64(np.ascontiguousarray(x).view(np.uint64), n, r, m, u)
            return u.view(np.int64)
        raise TypeError(x.dtype)

    def subspace_index(self, rows, kp: int) -> int:
        """A^T k' = XOR of rows[t] over the set bits t of k'."""
        r = np.ascontiguousarray(np.asarray(rows, dtype=np.uint64))
        return int(self._L.subspace_index(r, r.size, int(kp)))

    def subspace_indices(self, rows, kps) -> np.ndarray:
        return np.array([self.subspace_index(rows, k) for k in kps], dtype=np.uint64)

    # ---- prime-factor counts (the workload announced in section 4.3) --------
    def prime_omega(self, count: int, threads: int | None = None) -> np.ndarray:
        """Omega(i) (prime factors with multiplicity; Omega(0) = Omega(1) = 0)
        for i in [0, count), int32, on `threads` host threads."""
        out = np.empty(max(count, 1), dtype=np.int32)
        if self._L.prime_omega(count, out, threads or host_threads()) != 0:
            raise MemoryError("prime_omega")
        return out[:count]

    def prime_omega_at(self, ks) -> np.ndarray:
        """Omega(k) of single numbers by trial division."""
        return np.array([self._L.prime_omega_at(int(k)) for k in ks], dtype=np.int64)


    # ---- checks of transforms too large to keep an oracle copy of ------------
    KF_P = (1 << 61) - 1

    def kf_sum(self, data: np.ndarray, n: int, t, side: int, start: int = 0,
               threads: int | None = None) -> int:
        """sum_i data[i] * w(start + i) mod P = 2^61 - 1, for a slice of a
        transform of 2^n entries: side 0 weighs the output index k by
        prod_j t_j^(bit j of k), side 1 the input index i by
        prod_j (1 + (-1)^(bit j of i) t_j).  For a correct transform the two
        sides agree (H is symmetric); see ``kf_sum`` in wht_oracle.c."""
        data = np.ascontiguousarray(data)
        if data.dtype not in (np.int32, np.int64):
            raise TypeError(data.dtype)
        tv = np.ascontiguousarray(np.asarray(t, dtype=np.uint64))
        if tv.size < n:
            raise ValueError("t needs n entries")
        r = self._L.kf_sum(data.ctypes.data_as(C.c_void_p), data.itemsize, int(start), data.size, int(n), tv,
                           int(side), threads or host_threads())
        if r == (1 << 64) - 1:
            raise ValueError("kf_sum: bad arguments")
        return int(r)

    def sumsq(self, data: np.ndarray, mod_p: bool = False, threads: int | None = None) -> int:
        """sum of data[i]^2 mod 2^64 (wrap-around), or mod P = 2^61 - 1."""
        data = np.ascontiguousarray(data)
        if data.dtype not in (np.int32, np.int64):
            raise TypeError(data.dtype)
        return int(self._L.sumsq_mod(data.ctypes.data_as(C.c_void_p), data.itemsize, data.size, int(bool(mod_p)),
                                     threads or host_threads()))


def host_threads() -> int:
    """Threads the multi-threaded oracle functions use: the host's cores, at
    most 16."""
    return max(1, min(16, os.cpu_count() or 1))


# ---- GF(2) linear algebra for section 5.1 (plain Gaussian elimination) ------

def gf2_rank(rows) -> int:
    """Rank over GF(2) of the bit vectors `rows` (Python ints)."""
    basis = []  # rows with distinct leading (highest) bits
    for r in (int(v) for v in rows):
        for b in basis:
            r = min(r, r ^ b)
        if r:
            basis.append(r)
            basis.sort(reverse=True)
    return len(basis)


def gf2_canonical_rows(rows, n: int):
    """The unique reduced echelon basis of the row space of `rows` with
    pivots at the lowest bits: row t has its lowest set bit p_t, p_0 < p_1 <
    ..., and bit p_t is clear in every other row.  Returns a list of ints,
    or None when the rows are linearly dependent."""
    rs = [int(v) for v in rows]
    m = len(rs)
    if any(v >> n for v in rs):
        raise ValueError("row has bits at or above n")
    out = []
    rest = list(rs)
    for bit in range(n):
        piv = next((v for v in rest if (v >> bit) & 1), None)
        if piv is None:
            continue
        rest.remove(piv)
        rest = [v ^ piv if (v >> bit) & 1 else v for v in rest]
        out = [v ^ piv if (v >> bit) & 1 else v for v in out]
        out.append(piv)
    if len(out) < m:
        return None
    return sorted(out, key=lambda v: (v & -v))


def fold_preimage(rows, n: int, j: int):
    """Every i in [0, 2^n) with A i = j (bit t of A i is parity(rows[t] & i)),
    by solving the linear system: one solution plus the span of the null
    space.  Returns a sorted numpy uint64 array (2^(n - m) entries when A has
    full rank m)."""
    rs = [int(v) for v in rows]
    m = len(rs)
    # augmented system over the n unknown bits of i: rows[t] . i = bit t of j
    eqs = [(rs[t], (j >> t) & 1) for t in range(m)]
    pivots = []  # (column, row-vector, rhs)
    for col in range(n):
        k = next((q for q, (v, _) in enumerate(eqs) if (v >> col) & 1), None)
        if k is None:
            continue
        v, c = eqs.pop(k)
        eqs = [(w ^ v, d ^ c) if (w >> col) & 1 else (w, d) for (w, d) in eqs]
        pivots = [(pc, w ^ v, d ^ c) if (w >> col) & 1 else (pc, w, d) for (pc, w, d) in pivots]
        pivots.append((col, v, c))
    if any(d for (_, d) in eqs):
        return np.zeros(0, dtype=np.uint64)  # inconsistent (rank deficient)
    pcols = {pc for (pc, _, _) in pivots}
    free = [c for c in range(n) if c not in pcols]
    # each pivot variable equals its rhs plus the free variables in its row
    sols = []
    for fmask in range(1 << len(free)):
        i = 0
        for q, c in enumerate(free):
            if (fmask >> q) & 1:
                i |= 1 << c
        for (pc, v, d) in pivots:
            bit = d ^ (bin(v & i & ~(1 << pc)).count("1") & 1)
            i |= bit << pc
        sols.append(i)
    return np.array(sorted(sols), dtype=np.uint64)


def _log2(size: int) -> int:
    n = int(size).bit_length() - 1
    if size <= 0 or (1 << n) != size:
        raise ValueError(f"length {size} is not a power of two")
    return n


_default: Oracle | None = None


def get() -> Oracle:
    """The default (unmutated) oracle, built on first use."""
    global _default
    if _default is None:
        _default = Oracle(LIB)
    return _default
