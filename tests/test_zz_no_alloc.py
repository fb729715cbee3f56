"""The allocation-free batched entry point against the cached-graph one.

fwht_batched_noalloc runs the same persistent kernels as fwht_batched from a
work list in a fixed device array of the library, so on the same input both
must give the same bits; both are also held to the FP64 oracle's bound.  Two
calls in a row, the second with fewer and smaller transforms, check that the
array keeps nothing from one call to the next that matters.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import paper_1607_01039_amd as F  # an import failure fails collection, never skips
import synth
from paper_1607_01039_amd import _lib

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _native_library():
    assert torch.cuda.is_available()
    _lib.lib()


def _call(entry, t, off, lg, prec):
    L = _lib.lib()
    off = np.ascontiguousarray(off, dtype=np.int64)
    lg = np.ascontiguousarray(lg, dtype=np.int32)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = getattr(L, entry)(C.c_void_p(t.data_ptr()), off.ctypes.data_as(C.c_void_p), lg.ctypes.data_as(C.c_void_p),
                           len(off), 1, prec, stream)
    _lib.check(rc)


def _normwise_max(O, x, y, off, lg):
    ref = O.wht_ragged(x, off, lg, True)
    worst = 0.0
    for o, m in zip(off.tolist(), lg.tolist()):
        r = ref[o:o + (1 << m)]
        worst = max(worst, float(np.linalg.norm(y[o:o + (1 << m)] - r) / np.linalg.norm(r)))
    return worst


# (count, lo, hi, seed): the 4096-transform ragged workload, then a smaller
# second call with fewer, smaller transforms and other data
CALLS = [(4096, 8, 16, 4), (300, 2, 10, 9)]


@pytest.mark.parametrize("prec,bound", [(_lib.FWHT_PREC_FP32, None), (_lib.FWHT_PREC_FP16_MFMA, 1e-3)],
                         ids=["fp32", "fp16"])
def test_noalloc_matches_cached_entry_point(O, prec, bound):
    for count, lo, hi, seed in CALLS:
        print(f"no-alloc batched: prec={prec} count={count} sizes 2^{lo}..2^{hi}", flush=True)
        lg, off, tot = synth.ragged(count, lo, hi, seed)
        x = synth.normal(tot, seed)
        a = torch.from_numpy(x).cuda()
        b = a.clone()
        _call("fwht_batched", a, off, lg, prec)
        _call("fwht_batched_noalloc", b, off, lg, prec)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        y = b.cpu().numpy()
        err = _normwise_max(O, x, y, off, lg)
        limit = bound if bound is not None else 2 * (hi + 2) * 2.0 ** -23
        assert err <= limit, (count, err)


def test_noalloc_binding_and_repeat(O):
    # The Python name marshals to the same entry point; repeating a call on
    # the same array applies the transform again (orthonormal: twice = identity).
    lg, off, tot = synth.ragged(64, 2, 16, 12)
    x = synth.normal(tot, 12)
    t = torch.from_numpy(x).cuda()
    F.fwht_batched_noalloc_(t, off, lg)
    F.fwht_batched_noalloc_(t, off, lg)
    torch.cuda.synchronize()
    assert np.max(np.abs(t.cpu().numpy() - x)) <= 1e-5 * max(1.0, float(np.max(np.abs(x))))
