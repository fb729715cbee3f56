"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module generates signals only; it performs no Walsh-Hadamard arithmetic.
Every integer signal is a pure function of (seed, index), built from the
SplitMix64 generator of Steele, Lea and Flood ("Fast splittable pseudorandom
number generators", OOPSLA 2014): from a 64-bit state, each output adds the
golden-ratio increment 0x9E3779B97F4A7C15 and applies the finaliser

    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    z =  z ^ (z >> 31)

so output number i (0-based) of a stream with state S is mix(S + (i+1)*G).
A stream's state is itself output number `stream` of the generator seeded with
`seed`.  Any slice of any signal can therefore be regenerated on its own.

Signals (the workloads of the paper's setting, section 2: a +-1 signal, and a
Walsh function corrupted by i.i.d. noise):

* ``signs``   : x_i = 1 - 2 * (h_i >> 63)                 (stream 0)
* ``planted`` : s = low n bits of output 0 of stream 1;
                e_i = [(h_i >> 32) < floor(p * 2^32)]      (stream 2);
                x_i = (-1)^(popcount(s & i) xor e_i)
* float signals (N(0,1), U(0,1)) and ragged sizes come from numpy's PCG64
  with the given seed; they are generated once on the host and the same
  buffers are handed to both sides.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "synth.c")
LIB = os.path.join(HERE, "libsynth.so")
_lib = None


def build() -> str:
    """Compile the C generator (same definitions, multi-threaded)."""
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                    "-o", LIB, SRC], check=True)
    return LIB


def _clib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        L.synth_splitmix64.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, C.c_void_p]
        L.synth_signs.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, C.c_void_p, C.c_int]
        L.synth_planted.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64,
                                    C.c_uint64, C.c_void_p, C.c_int]
        L.synth_planted.restype = C.c_uint64
        _lib = L
    return _lib

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_CHUNK = 1 << 22


def _mix(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser on a uint64 array (in place, returned)."""
    z ^= z >> np.uint64(30)
    z *= _M1
    z ^= z >> np.uint64(27)
    z *= _M2
    z ^= z >> np.uint64(31)
    return z


def splitmix64(state: int, start: int, count: int) -> np.ndarray:
    """Outputs start .. start+count-1 of SplitMix64 begun from `state`."""
    with np.errstate(over="ignore"):
        i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(state & 0xFFFFFFFFFFFFFFFF) + i * GOLDEN
        return _mix(z)


def stream_state(seed: int, stream: int) -> int:
    """State of sub-stream `stream` of seed `seed`."""
    return int(splitmix64(seed, stream, 1)[0])


def _chunks(count: int):
    for c0 in range(0, count, _CHUNK):
        yield c0, min(_CHUNK, count - c0)


def signs_ref(count: int, seed: int, dtype=np.int32) -> np.ndarray:
    """Uniform random signs x_i in {+1, -1} (stream 0); numpy definition."""
    st = stream_state(seed, 0)
    out = np.empty(count, dtype=dtype)
    for c0, c in _chunks(count):
        h = splitmix64(st, c0, c)
        out[c0:c0 + c] = (1 - 2 * (h >> np.uint64(63)).astype(np.int64)).astype(dtype)
    return out


def bernoulli_threshold(p: float) -> int:
    """Integer threshold t with P[(h >> 32) < t] = t / 2^32, t = floor(p 2^32)."""
    return int(np.floor(p * 2.0 ** 32))


def planted_mask(n: int, seed: int) -> int:
    """The planted n-bit mask s (stream 1, output 0)."""
    return int(splitmix64(stream_state(seed, 1), 0, 1)[0]) & ((1 << n) - 1)


def planted_ref(n: int, seed: int, p: float, dtype=np.int32, start: int = 0,
                count: int | None = None):
    """Planted-peak signal, numpy definition (see ``planted``)."""
    N = 1 << n
    if count is None:
        count = N - start
    s = planted_mask(n, seed)
    st = stream_state(seed, 2)
    thr = np.uint64(bernoulli_threshold(p))
    out = np.empty(count, dtype=dtype)
    errors = 0
    su = np.uint64(s)
    for c0, c in _chunks(count):
        h = splitmix64(st, start + c0, c)
        e = (h >> np.uint64(32)) < thr
        errors += int(np.count_nonzero(e))
        i = np.arange(start + c0, start + c0 + c, dtype=np.uint64)
        par = (np.bitwise_count(i & su) & np.uint8(1)).astype(bool)
        neg = par ^ e
        out[c0:c0 + c] = np.where(neg, -1, 1).astype(dtype)
    return out, s, errors


def planted_params(n: int, seed: int, p: float):
    """(s, state, thr) of the planted signal: the mask, the state of the noise
    stream and the Bernoulli threshold, which together define x_i for any i
    (as an on-the-fly signal source regenerates it)."""
    return planted_mask(n, seed), stream_state(seed, 2), bernoulli_threshold(p)


def planted_at(n: int, seed: int, p: float, idx) -> np.ndarray:
    """The planted signal (int64) at arbitrary indices `idx`; numpy definition."""
    s, st, thr = planted_params(n, seed, p)
    i = np.ascontiguousarray(np.asarray(idx, dtype=np.uint64))
    with np.errstate(over="ignore"):
        h = _mix(np.uint64(st) + (i + np.uint64(1)) * GOLDEN)
    e = (h >> np.uint64(32)) < np.uint64(thr)
    par = (np.bitwise_count(i & np.uint64(s)) & np.uint8(1)).astype(bool)
    return np.where(par ^ e, -1, 1).astype(np.int64)


def subspace_rows(n: int, m: int, seed: int) -> np.ndarray:
    """m random n-bit rows (uint64, numpy PCG64) for a linear space reduction
    GF(2)^n -> GF(2)^m; redrawn until they are linearly independent."""
    rng = np.random.Generator(np.random.PCG64(seed))
    while True:
        rows = rng.integers(0, 1 << n, size=m, dtype=np.uint64) if n < 64 else \
            rng.integers(0, np.iinfo(np.uint64).max, size=m, dtype=np.uint64, endpoint=True)
        basis = []
        for r in (int(v) for v in rows):
            for b in basis:
                r = min(r, r ^ b)
            if r:
                basis.append(r)
                basis.sort(reverse=True)
        if len(basis) == m:
            return rows


def signs(count: int, seed: int, dtype=np.int32, start: int = 0) -> np.ndarray:
    """Uniform random signs x_i in {+1, -1} (stream 0), indices start..start+count-1."""
    out = np.empty(count, dtype=dtype)
    _clib().synth_signs(stream_state(seed, 0), start, count,
                        out.ctypes.data_as(C.c_void_p), out.itemsize)
    return out


def planted(n: int, seed: int, p: float, dtype=np.int32, start: int = 0,
            count: int | None = None, out: np.ndarray | None = None):
    """Planted-peak signal x_i = (-1)^(popcount(s & i) xor e_i), e_i ~ Bern(p).

    Returns (x, s, errors) where `errors` counts the e_i = 1 in the slice.
    """
    N = 1 << n
    if count is None:
        count = N - start
    if out is None:
        out = np.empty(count, dtype=dtype)
    assert out.size == count and out.flags.c_contiguous
    s = planted_mask(n, seed)
    errors = _clib().synth_planted(stream_state(seed, 2), s, bernoulli_threshold(p),
                                   start, count, out.ctypes.data_as(C.c_void_p),
                                   out.itemsize)
    return out, s, int(errors)


def raw64(count: int, seed: int, out: np.ndarray | None = None) -> np.ndarray:
    """Full-range int64 values: the SplitMix64 outputs of stream 3, read as
    two's-complement (every bit of a 64-bit word random, so transforms of
    them wrap around mod 2^64 at every size)."""
    if out is None:
        out = np.empty(count, dtype=np.int64)
    assert out.size == count and out.dtype == np.int64 and out.flags.c_contiguous
    _clib().synth_splitmix64(stream_state(seed, 3), 0, count, out.ctypes.data_as(C.c_void_p))
    return out


def normal(shape, seed: int) -> np.ndarray:
    """i.i.d. N(0,1) float32 (numpy PCG64)."""
    return np.random.Generator(np.random.PCG64(seed)).standard_normal(shape, dtype=np.float32)


def uniform(shape, seed: int) -> np.ndarray:
    """i.i.d. U(0,1) float32 (numpy PCG64)."""
    return np.random.Generator(np.random.PCG64(seed)).random(shape, dtype=np.float32)


def ragged(count: int, lo: int, hi: int, seed: int):
    """Sizes n_t ~ U{lo..hi} and packed offsets for `count` transforms.

    Returns (log2n int32[count], offsets int64[count], total elements).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    lg = rng.integers(lo, hi + 1, size=count).astype(np.int32)
    sizes = np.left_shift(np.int64(1), lg.astype(np.int64))
    off = np.zeros(count, dtype=np.int64)
    if count > 1:
        off[1:] = np.cumsum(sizes)[:-1]
    return lg, off, int(sizes.sum())


def ints(count: int, seed: int, lo: int, hi: int, dtype=np.int64) -> np.ndarray:
    """Uniform integers in [lo, hi] (numpy PCG64), for exactness tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(lo, hi + 1, size=count, dtype=np.int64).astype(dtype)
