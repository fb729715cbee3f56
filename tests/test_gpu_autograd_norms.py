"""GPU: the differentiable transform (autograd) and the FP64 norm reductions.

Gradient of L = sum_{b,k} w_bk (Y x_b)_k^2 with Y = 2^(-n/2) H: the oracle's
closed form 2 Y (w * Y x) in FP64, and central finite differences (eps = 1e-3,
FP64 per-row loss; the loss is quadratic so the difference quotient is exact
up to rounding).  Tolerance 1e-4, the bound stated for this workload.
"""
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


def test_autograd_matches_oracle_gradient(F, O):
    import torch
    n, B = 12, 8
    x = synth.normal((B, 1 << n), 5)
    w = synth.uniform((B, 1 << n), 6)
    xt = torch.from_numpy(x).cuda().requires_grad_(True)
    wt = torch.from_numpy(w).cuda()
    y = F.fwht(xt)
    loss = (wt * y * y).sum()
    loss.backward()
    g = xt.grad.cpu().numpy().astype(np.float64)
    gref = O.grad_weighted_square(x, w, n)
    rel = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    assert rel <= 1e-4, rel
    # forward equals the orthonormal oracle
    yref = O.wht_batch(x, n, True)
    assert np.linalg.norm(y.detach().cpu().numpy() - yref) / np.linalg.norm(yref) <= 1e-6


def test_autograd_config_256x2p20_fd_and_oracle(F, O):
    """256 x 2^20, x ~ N(0,1), w ~ U(0,1) (seed 5): gradient on the GPU, checked
    on sampled rows against the oracle gradient and, along sampled
    directions inside a row, against central differences of the FP64 loss."""
    import torch
    n, B = 20, 256
    x = synth.normal((B, 1 << n), 5)
    w = synth.uniform((B, 1 << n), 55)
    xt = torch.from_numpy(x).cuda().requires_grad_(True)
    wt = torch.from_numpy(w).cuda()
    y = F.fwht(xt)
    (wt * y * y).sum().backward()
    g = xt.grad.cpu().numpy()
    del xt, wt, y
    torch.cuda.empty_cache()
    rng = np.random.default_rng(1)
    for row in (0, 131, 255):
        xr = x[row:row + 1].astype(np.float64)
        wr = w[row:row + 1].astype(np.float64)
        gref = O.grad_weighted_square(xr, wr, n)
        rel = np.linalg.norm(g[row] - gref[0]) / np.linalg.norm(gref)
        assert rel <= 1e-4, (row, rel)

        def loss(z):
            yz = O.wht_batch(z, n, True)
            return float(np.sum(wr * yz * yz))

        eps = 1e-3
        for _ in range(2):
            v = rng.standard_normal(xr.shape)
            fd = (loss(xr + eps * v) - loss(xr - eps * v)) / (2 * eps)
            an = float(np.sum(g[row].astype(np.float64) * v[0]))
            assert abs(an - fd) / abs(fd) <= 1e-4, (row, an, fd)


def test_backward_is_the_same_kernel(F):
    import torch
    n = 10
    x = torch.from_numpy(synth.normal((3, 1 << n), 9)).cuda().requires_grad_(True)
    g = torch.from_numpy(synth.normal((3, 1 << n), 10)).cuda()
    y = F.fwht(x)
    y.backward(g)
    direct = g.clone()
    F.fwht_float_(direct)
    assert torch.equal(x.grad, direct)


def test_norms_fp64(F, O):
    import torch
    lg, off, tot = synth.ragged(37, 2, 16, 11)
    x = synth.normal(tot, 1)
    xt = torch.from_numpy(x).cuda()
    yt = xt.clone()
    for t in range(37):
        seg = yt[off[t]:off[t] + (1 << int(lg[t]))]
        F.fwht_float_(seg.view(1, -1))
    y = yt.cpu().numpy()
    r = O.wht_ragged(x, off, lg, True)
    out = F.norms(xt, yt, off, lg, r=torch.from_numpy(r).cuda()).cpu().numpy()
    sx, sy, se = O.norms(x, y, r, off, lg)
    assert np.allclose(out[:, 0], sx, rtol=1e-12)
    assert np.allclose(out[:, 1], sy, rtol=1e-12)
    assert np.allclose(out[:, 2], se, rtol=1e-9, atol=1e-300)
    # Parseval: the orthonormal transform keeps the sum of squares
    assert np.allclose(out[:, 1], out[:, 0], rtol=1e-5)
    out0 = F.norms(xt, yt, off, lg).cpu().numpy()
    assert np.all(out0[:, 2] == 0.0)


def test_norms_unaligned_and_large(F, O):
    """Transforms of 1, 2 and 8 entries at offsets that are not multiples of 4
    (the scalar path), next to one of 2^22 entries cut into 1024 chunks (the
    vector path), against the oracle's FP64 sums."""
    import torch
    lg = np.array([0, 1, 3, 22, 1, 0, 5], dtype=np.int32)
    sizes = np.left_shift(np.int64(1), lg.astype(np.int64))
    off = np.zeros(len(lg), dtype=np.int64)
    off[1:] = np.cumsum(sizes)[:-1]
    tot = int(sizes.sum())
    x = synth.normal(tot, 21)
    y = synth.normal(tot, 22)
    r = synth.normal(tot, 23).astype(np.float64)
    out = F.norms(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), off, lg,
                  r=torch.from_numpy(r).cuda()).cpu().numpy()
    sx, sy, se = O.norms(x, y, r, off, lg)
    assert np.allclose(out[:, 0], sx, rtol=1e-12)
    assert np.allclose(out[:, 1], sy, rtol=1e-12)
    assert np.allclose(out[:, 2], se, rtol=1e-12)



def test_norms_same_request_two_streams(F, O):
    """Calls of one request share its buffer of partial sums: back-to-back calls
    on two streams, each with inputs of its own and an FP64 reference, must both
    match the oracle (the second waits on the GPU for the first)."""
    import torch
    lg, off, tot = synth.ragged(64, 8, 16, 12)
    xs = [synth.normal(tot, 31 + k) for k in range(3)]
    ys = [synth.normal(tot, 41 + k) for k in range(3)]
    rs = [synth.normal(tot, 51 + k).astype(np.float64) for k in range(3)]
    xt = [torch.from_numpy(a).cuda() for a in xs]
    yt = [torch.from_numpy(a).cuda() for a in ys]
    rt = [torch.from_numpy(a).cuda() for a in rs]
    streams = [torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.current_stream()]
    torch.cuda.synchronize()
    outs = []
    for k, st in enumerate(streams):
        with torch.cuda.stream(st):
            outs.append(F.norms(xt[k], yt[k], off, lg, r=rt[k]))
    torch.cuda.synchronize()
    for k in range(3):
        sx, sy, se = O.norms(xs[k], ys[k], rs[k], off, lg)
        got = outs[k].cpu().numpy()
        assert np.allclose(got[:, 0], sx, rtol=1e-12)
        assert np.allclose(got[:, 1], sy, rtol=1e-12)
        assert np.allclose(got[:, 2], se, rtol=1e-12)
