"""MI355X-native Walsh-Hadamard transform (Lu, arXiv 1607.01039).

Python surface over the C ABI of ``libfwht.so`` (include/fwht.h).  torch is
used for device memory and streams only; every transform, threshold pass and
reduction runs in the library's HIP kernels.

* ``fwht_int_(t, threshold=None, cap=...)`` -- in-place integer WHT (section 2,
  Eq. 2) of a 1-D int32/int64 CUDA tensor of 2^n entries, optionally with the
  fused pass returning every (k, W_k) with |W_k| > T, or of a pinned host
  int64 tensor (streamed path, synchronous).
* ``fwht_float_(t, normalize=True, precision="fp32")`` -- in-place float WHT
  over the last dimension (2^n) of a float32 CUDA tensor.
* ``fwht_batched_(data, offsets, log2n, ...)`` -- uneven batched transforms in
  one persistent launch replayed from a cached HIP graph.
* ``threshold(t, T, cap)`` -- stand-alone threshold pass.
* ``fwht(x)`` -- differentiable orthonormal transform (autograd Function whose
  backward is the same self-adjoint kernel).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import FWHTError

PRECISIONS = {"fp32": _lib.FWHT_PREC_FP32, "fp16": _lib.FWHT_PREC_FP16_MFMA,
              "bf16": _lib.FWHT_PREC_BF16_MFMA}

__all__ = ["fwht_int_", "hit_buffers", "fwht_float_", "fwht_float_out", "fwht_batched_", "fwht_batched_noalloc_",
           "threshold", "fwht", "FWHTFunction", "norms", "set_schedule", "get_schedule", "set_batched_tiles", "get_batched_tiles", "set_batched_graphs",
           "get_batched_graphs", "trace_enable",
           "trace_read", "copy_",
           "fold_", "fold_planted", "subspace_hits_", "subspace_transform", "subspace_scan", "prime_omega",
           "FWHTError", "PRECISIONS"]


def _torch():
    import torch
    return torch


def _stream_ptr(t=None):
    torch = _torch()
    if t is not None and not t.is_cuda:
        return None
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _log2(size: int) -> int:
    n = int(size).bit_length() - 1
    if size <= 0 or (1 << n) != size:
        raise ValueError(f"length {size} is not a power of two")
    return n


class Hits:
    """Result of a threshold pass: indices and values of the hits (sorted by
    index on request) plus the true count."""

    def __init__(self, idx, val, count, cap):
        self.idx, self.val, self.count, self.cap = idx, val, count, cap

    @property
    def overflow(self) -> bool:
        return self.count > self.cap

    def sorted(self):
        order = np.argsort(self.idx, kind="stable")
        return self.idx[order], self.val[order]


def _thresh_buffers(dtype, cap, device):
    """(idx, val, count) output buffers of a threshold request; the library
    clears the count itself, so nothing is initialised here."""
    torch = _torch()
    idx = torch.empty(max(cap, 1), dtype=torch.int64, device=device)
    val = torch.empty(max(cap, 1), dtype=dtype, device=device)
    cnt = torch.empty(1, dtype=torch.int64, device=device)
    return idx, val, cnt


def hit_buffers(t, cap: int = 1 << 16):
    """Reusable output buffers for ``fwht_int_(t, threshold=..., hits=...)``
    (a call that passes them allocates nothing)."""
    return _thresh_buffers(t.dtype, cap, t.device)


def _collect(idx, val, cnt, cap) -> Hits:
    count = int(cnt.cpu().item())
    k = min(count, cap)
    return Hits(idx[:k].cpu().numpy().view(np.uint64).astype(np.int64), val[:k].cpu().numpy(), count, cap)


def fwht_int_(t, threshold=None, cap: int = 1 << 16, sync: bool = True, hits=None):
    """In-place unnormalised integer WHT of a 1-D int32 / int64 tensor of 2^n entries.

    With ``threshold=T`` the last pass also collects every (k, W_k) with
    |W_k| > T; returns a ``Hits`` (after a stream sync when ``sync``), else
    the (idx, val, count) buffers.  ``hits`` may pass buffers from
    ``hit_buffers`` (device tensors; their capacity replaces ``cap``).  A
    pinned host int64 tensor runs the streamed path synchronously.
    """
    torch = _torch()
    if t.dim() != 1 or not t.is_contiguous():
        raise ValueError("fwht_int_ needs a contiguous 1-D tensor")
    dt = {torch.int32: _lib.FWHT_I32, torch.int64: _lib.FWHT_I64}.get(t.dtype)
    if dt is None:
        raise TypeError("fwht_int_ needs int32 or int64")
    n = _log2(t.numel())
    L = _lib.lib()
    th = None
    bufs = None
    if threshold is not None:
        device = t.device if t.is_cuda else "cpu"
        if hits is not None:
            if not t.is_cuda:
                raise ValueError("hits buffers are for device tensors")
            bufs = hits
            cap = int(hits[0].numel())
        elif t.is_cuda:
            bufs = _thresh_buffers(t.dtype, cap, device)
        else:
            bufs = tuple(b.pin_memory() for b in _thresh_buffers(t.dtype, cap, "cpu"))
        th = _lib.fwht_thresh_t(int(threshold), 0.0, bufs[0].data_ptr(), bufs[1].data_ptr(), cap,
                                bufs[2].data_ptr())
    stream = _stream_ptr(t) if t.is_cuda else C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.fwht_int(C.c_void_p(t.data_ptr()), dt, n, C.byref(th) if th else None, stream)
    if rc == _lib.FWHT_E_CAPACITY and bufs is not None:
        return _collect(*bufs, cap)
    _lib.check(rc)
    if bufs is None:
        return None
    if not sync:
        return bufs
    if t.is_cuda:
        torch.cuda.current_stream().synchronize()
    return _collect(*bufs, cap)


# ---- section 5.1: linear space reduction -------------------------------------

def _rows_array(rows, m):
    r = np.ascontiguousarray(np.asarray(rows, dtype=np.uint64).reshape(-1))
    if r.size != m:
        raise ValueError(f"expected {m} rows, got {r.size}")
    return r


def fold_(x, m: int, rows, out=None):
    """Reduce a stored signal (1-D int32/int64 CUDA tensor of 2^n entries) by the
    linear map A : GF(2)^n -> GF(2)^m with the given rows (bit t of A i is the
    parity of rows[t] & i): u_j = sum of x_i over A i = j.  Returns (u, basis):
    u (2^m entries, x's dtype) is the reduction by the canonical basis of the
    row space, and entry k' of u's transform is the coefficient of x at the
    XOR of basis[t] over the set bits t of k'."""
    torch = _torch()
    if x.dim() != 1 or not x.is_contiguous() or not x.is_cuda:
        raise ValueError("fold_ needs a contiguous 1-D CUDA tensor")
    dt = {torch.int32: _lib.FWHT_I32, torch.int64: _lib.FWHT_I64}.get(x.dtype)
    if dt is None:
        raise TypeError("fold_ needs int32 or int64")
    n = _log2(x.numel())
    r = _rows_array(rows, m)
    if out is None:
        out = torch.empty(1 << m, dtype=x.dtype, device=x.device)
    if out.numel() != 1 << m or out.dtype != x.dtype or not out.is_contiguous():
        raise ValueError("out must be a contiguous tensor of 2^m entries of x's dtype")
    basis = np.zeros(max(m, 1), dtype=np.uint64)
    _lib.check(_lib.lib().fwht_fold(C.c_void_p(x.data_ptr()), dt, n, m, r.ctypes.data_as(C.c_void_p),
                                    C.c_void_p(out.data_ptr()), basis.ctypes.data_as(C.c_void_p),
                                    _stream_ptr(x)))
    return out, basis[:m]


def fold_planted(n: int, m: int, rows, mask: int, state: int, thr: int, dtype=None, out=None,
                 device="cuda"):
    """Reduce the planted signal x_i = (-1)^(<mask, i> xor [(h_i >> 32) < thr])
    (h_i: SplitMix64 output i of the stream with `state`), generated on the fly
    inside the reduction, to 2^m entries.  Returns (u, basis) as ``fold_``."""
    torch = _torch()
    dtype = torch.int64 if dtype is None else dtype
    dt = {torch.int32: _lib.FWHT_I32, torch.int64: _lib.FWHT_I64}.get(dtype)
    if dt is None:
        raise TypeError("fold_planted needs int32 or int64")
    r = _rows_array(rows, m)
    if out is None:
        out = torch.empty(1 << m, dtype=dtype, device=device)
    if out.numel() != 1 << m or out.dtype != dtype or not out.is_contiguous() or not out.is_cuda:
        raise ValueError("out must be a contiguous CUDA tensor of 2^m entries of `dtype`")
    basis = np.zeros(max(m, 1), dtype=np.uint64)
    _lib.check(_lib.lib().fwht_fold_planted(dt, n, m, r.ctypes.data_as(C.c_void_p), int(mask), int(state),
                                            int(thr), C.c_void_p(out.data_ptr()),
                                            basis.ctypes.data_as(C.c_void_p), _stream_ptr(out)))
    return out, basis[:m]


def subspace_hits_(bufs, basis) -> None:
    """Map the hit indices k' of a threshold on a reduced transform, in the
    device buffers (idx, val, count) from ``fwht_int_(..., sync=False)``, to
    the full-space indices (XOR of basis[t] over the set bits t of k')."""
    idx, _, cnt = bufs
    b = np.ascontiguousarray(np.asarray(basis, dtype=np.uint64))
    _lib.check(_lib.lib().fwht_subspace_hits(C.c_void_p(idx.data_ptr()), int(idx.numel()),
                                             C.c_void_p(cnt.data_ptr()), int(b.size),
                                             b.ctypes.data_as(C.c_void_p), _stream_ptr(idx)))


def subspace_transform(u, basis, threshold, cap: int = 1 << 16, hits=None) -> Hits:
    """Transform a reduced signal u in place (2^m-point WHT) and return the
    coefficients above ``threshold`` with their full-space indices."""
    bufs = fwht_int_(u, threshold=threshold, cap=cap, sync=False, hits=hits)
    cap = int(bufs[0].numel())
    subspace_hits_(bufs, basis)
    _torch().cuda.current_stream().synchronize()
    return _collect(*bufs, cap)


def subspace_scan(source, m: int, rows_list, threshold, cap: int = 1 << 16, dtype=None):
    """Section 5.1's scheme of independent reductions (one per machine in the
    paper) run one after another on this GPU: each rank-m reduction in
    ``rows_list`` (caller-drawn rows) of the same signal is transformed and
    thresholded, and the hits are merged by full-space index.

    ``source`` is a stored signal (1-D int32/int64 CUDA tensor) or the planted
    signal's parameters ``(n, mask, state, thr)`` generated on the fly.
    Returns ``(hits, bases)``: a dict {index: coefficient} of every coefficient
    above ``threshold`` on the union of the subspaces, and the canonical basis
    of each reduction (the subspaces it covered)."""
    torch = _torch()
    out, bufs, hits, bases = None, None, {}, []
    for rows in rows_list:
        if isinstance(source, tuple):
            n, mask, state, thr = source
            out, basis = fold_planted(n, m, rows, mask, state, thr, dtype=dtype, out=out)
        else:
            out, basis = fold_(source, m, rows, out=out)
        if bufs is None:
            bufs = hit_buffers(out, cap)
        h = subspace_transform(out, basis, threshold, hits=bufs)
        if h.overflow:
            raise FWHTError(_lib.FWHT_E_CAPACITY, f"{h.count} hits exceed the capacity {cap}")
        for k, v in zip(h.idx.tolist(), h.val.tolist()):
            hits[int(k)] = int(v)
        bases.append(basis)
    return hits, bases


def prime_omega(n: int, dtype=None, out=None, device="cuda"):
    """The prime-factor-count signal Omega(i), i in [0, 2^n) (prime factors with
    multiplicity; Omega(0) = Omega(1) = 0), computed on the GPU (int64 by
    default: its transform exceeds int32 from n = 29)."""
    torch = _torch()
    dtype = torch.int64 if dtype is None else dtype
    dt = {torch.int32: _lib.FWHT_I32, torch.int64: _lib.FWHT_I64}.get(dtype)
    if dt is None:
        raise TypeError("prime_omega needs int32 or int64")
    if out is None:
        out = torch.empty(1 << n, dtype=dtype, device=device)
    if out.numel() != 1 << n or out.dtype != dtype or not out.is_contiguous() or not out.is_cuda:
        raise ValueError("out must be a contiguous CUDA tensor of 2^n entries of `dtype`")
    _lib.check(_lib.lib().fwht_prime_omega(C.c_void_p(out.data_ptr()), dt, n, _stream_ptr(out)))
    return out


def fwht_float_(t, normalize: bool = True, precision: str = "fp32"):
    """In-place float WHT over the last dimension (2^n) of a float32 CUDA tensor."""
    torch = _torch()
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise TypeError("fwht_float_ needs a contiguous float32 CUDA tensor")
    n = _log2(t.shape[-1])
    batch = t.numel() >> n
    _lib.check(_lib.lib().fwht_float(C.c_void_p(t.data_ptr()), n, batch, int(bool(normalize)),
                                     PRECISIONS[precision], _stream_ptr(t)))
    return t


def fwht_float_out(src, out=None, normalize: bool = True, precision: str = "fp32"):
    """Out-of-place float WHT over the last dimension: returns ``out`` (a new
    tensor if None) holding the transform of ``src``, which is left unchanged."""
    torch = _torch()
    if src.dtype != torch.float32 or not src.is_cuda or not src.is_contiguous():
        raise TypeError("fwht_float_out needs a contiguous float32 CUDA tensor")
    if out is None:
        out = torch.empty_like(src)
    elif out.shape != src.shape or out.dtype != src.dtype or not out.is_contiguous() or out.device != src.device:
        raise TypeError("out must be a contiguous float32 tensor of src's shape on its device")
    n = _log2(src.shape[-1])
    batch = src.numel() >> n
    _lib.check(_lib.lib().fwht_float_out(src.data_ptr(), out.data_ptr(), n, batch, int(bool(normalize)),
                                         PRECISIONS[precision], _stream_ptr(src)))
    return out


def fwht_batched_(data, offsets, log2n, normalize: bool = True, precision: str = "fp32"):
    """In-place WHT of uneven transforms packed in a float32 CUDA tensor.

    ``offsets`` (int64) and ``log2n`` (int32) are host arrays (numpy or CPU
    tensors): transform t is data[offsets[t] : offsets[t] + 2^log2n[t]].
    """
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    lg = np.ascontiguousarray(log2n, dtype=np.int32)
    if off.shape != lg.shape:
        raise ValueError("offsets and log2n must have the same length")
    # raw addresses (ctypes' data_as costs microseconds per call)
    _lib.check(_lib.lib().fwht_batched(data.data_ptr(), off.ctypes.data, lg.ctypes.data, len(off),
                                       int(bool(normalize)), PRECISIONS[precision], _stream_ptr(data)))
    return data


def fwht_batched_noalloc_(data, offsets, log2n, normalize: bool = True, precision: str = "fp32"):
    """``fwht_batched_`` through the entry point that allocates nothing (a
    fixed work-list array of the library per GPU; at most 65536 transforms;
    calls on one GPU must not overlap)."""
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    lg = np.ascontiguousarray(log2n, dtype=np.int32)
    if off.shape != lg.shape:
        raise ValueError("offsets and log2n must have the same length")
    _lib.check(_lib.lib().fwht_batched_noalloc(data.data_ptr(), off.ctypes.data, lg.ctypes.data, len(off),
                                               int(bool(normalize)), PRECISIONS[precision], _stream_ptr(data)))
    return data


def threshold(t, T, cap: int = 1 << 16, hits=None, sync: bool = True):
    """Stand-alone pass: every (k, t[k]) with |t[k]| > T over a 1-D CUDA tensor
    of 2^n entries.  Returns a ``Hits`` after a stream sync when ``sync``, else
    the (idx, val, count) device buffers; ``hits`` may pass buffers from
    ``hit_buffers`` (their capacity replaces ``cap``)."""
    torch = _torch()
    dt = {torch.int32: _lib.FWHT_I32, torch.int64: _lib.FWHT_I64, torch.float32: _lib.FWHT_F32}[t.dtype]
    n = _log2(t.numel())
    if hits is not None:
        idx, val, cnt = hits
        cap = int(idx.numel())
    else:
        idx, val, cnt = _thresh_buffers(t.dtype, cap, t.device)
    if dt == _lib.FWHT_F32:
        th = _lib.fwht_thresh_t(0, float(T), idx.data_ptr(), val.data_ptr(), cap, cnt.data_ptr())
    else:
        th = _lib.fwht_thresh_t(int(T), 0.0, idx.data_ptr(), val.data_ptr(), cap, cnt.data_ptr())
    _lib.check(_lib.lib().fwht_threshold(C.c_void_p(t.data_ptr()), dt, n, C.byref(th), _stream_ptr(t)))
    if not sync:
        return idx, val, cnt
    torch.cuda.current_stream().synchronize()
    return _collect(idx, val, cnt, cap)


def norms(x, y, offsets, log2n, r=None):
    """FP64 per-transform (sum x^2, sum y^2, sum (y - r)^2) on the GPU -> (count, 3) float64 tensor."""
    torch = _torch()
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    lg = np.ascontiguousarray(np.asarray(log2n, dtype=np.int32))
    out = torch.empty((len(off), 3), dtype=torch.float64, device=x.device)
    # raw addresses: ctypes converts the ints itself, faster than explicit casts
    _lib.check(_lib.lib().fwht_norms(x.data_ptr(), y.data_ptr(), r.data_ptr() if r is not None else None,
                                     off.ctypes.data, lg.ctypes.data, len(off), out.data_ptr(), _stream_ptr(x)))
    return out


def trace_enable(on: bool = True) -> None:
    """Record a HIP event around every pass of later fwht_int_/fwht_float_ calls."""
    _lib.check(_lib.lib().fwht_trace_enable(int(bool(on))))


def trace_read():
    """[(pass name, device ms)] of the most recent traced call."""
    ms = (C.c_float * 64)()
    cnt = C.c_int(0)
    names = C.create_string_buffer(4096)
    _lib.check(_lib.lib().fwht_trace_read(ms, 64, C.byref(cnt), names, 4096))
    nm = names.value.decode().split(",") if cnt.value else []
    return list(zip(nm, [float(ms[i]) for i in range(cnt.value)]))


def copy_(dst, src) -> None:
    """Plain device copy kernel (reference kernel for bandwidth calibration)."""
    nbytes = src.numel() * src.element_size()
    _lib.check(_lib.lib().fwht_copy(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), nbytes,
                                    _stream_ptr(src)))


def set_schedule(dtype: str, n: int, spec):
    dt = {"int32": _lib.FWHT_I32, "int64": _lib.FWHT_I64, "float32": _lib.FWHT_F32}[dtype]
    _lib.check(_lib.lib().fwht_set_schedule(dt, n, spec.encode() if spec else None))


def list_variants(dtype: str):
    """Names of the compiled pass variants for `dtype`."""
    dt = {"int32": _lib.FWHT_I32, "int64": _lib.FWHT_I64, "float32": _lib.FWHT_F32}[dtype]
    buf = C.create_string_buffer(4096)
    _lib.check(_lib.lib().fwht_list_variants(dt, buf, 4096))
    return buf.value.decode().split(",")


def get_schedule(dtype: str, n: int) -> str:
    dt = {"int32": _lib.FWHT_I32, "int64": _lib.FWHT_I64, "float32": _lib.FWHT_F32}[dtype]
    buf = C.create_string_buffer(256)
    _lib.check(_lib.lib().fwht_get_schedule(dt, n, buf, 256))
    return buf.value.decode()


def set_batched_tiles(precision: str, spec):
    """Tile groups of the batched transform, e.g. "16:16,15:2-15"; None
    restores the tuned default."""
    _lib.check(_lib.lib().fwht_set_batched_tiles(PRECISIONS[precision], spec.encode() if spec else None))


def get_batched_tiles(precision: str = "fp32") -> str:
    buf = C.create_string_buffer(256)
    _lib.check(_lib.lib().fwht_get_batched_tiles(PRECISIONS[precision], buf, 256))
    return buf.value.decode()


def set_batched_graphs(on: bool) -> None:
    """Issue cached batched requests as HIP graph replays (True) or as direct
    launches of their work list (False, the default)."""
    _lib.check(_lib.lib().fwht_set_batched_graphs(int(bool(on))))


def get_batched_graphs() -> bool:
    return bool(_lib.lib().fwht_get_batched_graphs())


def _make_function():
    torch = _torch()

    class FWHTFunction(torch.autograd.Function):
        """Orthonormal WHT over the last dimension.  Y = 2^(-n/2) H is symmetric
        and orthogonal, so the adjoint applied in backward is Y itself: the
        same kernel runs on the incoming gradient."""

        @staticmethod
        def forward(ctx, x, precision="fp32"):
            ctx.precision = precision
            return fwht_float_out(x.contiguous(), None, True, precision)

        @staticmethod
        def backward(ctx, g):
            return fwht_float_out(g.contiguous(), None, True, ctx.precision), None

    return FWHTFunction


_fn = None


def __getattr__(name):
    global _fn
    if name == "FWHTFunction":
        if _fn is None:
            _fn = _make_function()
        return _fn
    raise AttributeError(name)


def fwht(x, precision: str = "fp32"):
    """Differentiable orthonormal WHT over the last dimension of a float32 CUDA tensor."""
    return __getattr__("FWHTFunction").apply(x, precision)
