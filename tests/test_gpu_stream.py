"""GPU parity of the streamed Kronecker path (pinned host arrays).

Small chunks (FWHT_STREAM_CHUNK_BYTES) force many row and column chunks
through the three-buffer pipeline; results must equal the oracle bit for
bit, also at the largest size with the default chunks (n = 32).
"""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available()
    import paper_1607_01039_amd as F
    F._lib.lib()
    return F


@pytest.fixture
def small_chunks():
    old = os.environ.get("FWHT_STREAM_CHUNK_BYTES")
    os.environ["FWHT_STREAM_CHUNK_BYTES"] = "4096"
    yield
    if old is None:
        del os.environ["FWHT_STREAM_CHUNK_BYTES"]
    else:
        os.environ["FWHT_STREAM_CHUNK_BYTES"] = old


def pinned(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).pin_memory()


@pytest.mark.parametrize("n", [10, 11, 16, 19, 22])
@pytest.mark.parametrize("dtype", [np.int64, np.int32])
def test_streamed_matches_oracle(F, O, small_chunks, n, dtype):
    lim = 1 << 40 if dtype == np.int64 else 1 << 8
    x = synth.ints(1 << n, 70 + n, -lim, lim, dtype=dtype)
    t = pinned(x)
    F.fwht_int_(t)
    assert np.array_equal(t.numpy(), O.wht_fig1(x))


@pytest.mark.parametrize("n,p,seed", [(16, 0.45, 3), (21, 0.48, 4)])
def test_streamed_threshold(F, O, small_chunks, n, p, seed):
    x, s, err = synth.planted(n, seed, p, dtype=np.int64)
    T = int(np.ceil(6 * 2 ** (n / 2))) // 2
    t = pinned(x)
    hits = F.fwht_int_(t, threshold=T, cap=1 << 14)
    ref = O.wht_fig1(x)
    assert np.array_equal(t.numpy(), ref)
    ridx, rval, rcnt = O.threshold(ref, T)
    gi, gv = hits.sorted()
    assert hits.count == rcnt and np.array_equal(gi, ridx.astype(np.int64)) and np.array_equal(gv, rval)
    assert s in set(gi.tolist())


def test_streamed_capacity(F, O, small_chunks):
    n = 14
    x = synth.signs(1 << n, 5, dtype=np.int64)
    t = pinned(x)
    hits = F.fwht_int_(t, threshold=-1, cap=50)
    assert hits.count == 1 << n and hits.overflow and len(hits.idx) == 50
    ref = O.wht_fig1(x)
    assert np.array_equal(ref[hits.idx], hits.val)


def test_streamed_equals_in_hbm_n28(F):
    """Default 1 GiB chunks, 2 GiB array: the streamed and in-HBM results agree."""
    import torch
    n = 28
    x = synth.ints(1 << n, 9, -(1 << 30), 1 << 30, dtype=np.int64)
    t = pinned(x)
    d = torch.from_numpy(x).cuda()
    F.fwht_int_(t)
    F.fwht_int_(d)
    torch.cuda.synchronize()
    assert torch.equal(t, d.cpu())


def test_streamed_planted_n32(F, O):
    """Planted peak at n = 32 (32 GiB of int64 in pinned host memory, p = 0.48,
    T = ceil(6 * 2^16)), default 1 GiB chunks: every entry against the
    oracle's Fig. 2 run on a host copy of the input, the hit set against the
    oracle's threshold scan, the closed-form peak, and the definition at the
    peak and at one other hit."""
    import torch
    n = 32
    N = 1 << n
    T = int(np.ceil(6 * 2 ** (n / 2)))
    print("streamed n=32: generating", flush=True)
    t = torch.empty(N, dtype=torch.int64, pin_memory=True)
    x, s, err = synth.planted(n, 3, 0.48, dtype=np.int64, out=t.numpy())
    ref = x.copy()
    print("streamed n=32: transforming", flush=True)
    hits = F.fwht_int_(t, threshold=T, cap=1 << 16)
    y = t.numpy()
    assert int(y[s]) == N - 2 * err
    gi, gv = hits.sorted()
    assert s in set(gi.tolist())
    other = [k for k in gi.tolist() if k != s][:1]
    print("streamed n=32: definition at sampled hits", flush=True)
    ks = [s] + other
    assert np.array_equal(O.wht_def_at(ref, ks), y[ks])
    print("streamed n=32: oracle (Fig. 2, 16 threads)", flush=True)
    O.wht_fig2_inplace(ref, 4)
    C = 1 << 27
    for c0 in range(0, N, C):
        assert np.array_equal(y[c0:c0 + C], ref[c0:c0 + C]), c0
    ridx, rval, rcnt = O.threshold(ref, T, cap=1 << 16)
    assert hits.count == rcnt and np.array_equal(gi, ridx.astype(np.int64)) and np.array_equal(gv, rval)
