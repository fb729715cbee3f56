"""Section 5.1 linear space reduction on the GPU against the oracle.

The library reduces by the canonical (reduced echelon, lowest-bit pivots)
basis of the caller's row space; the basis it returns must equal the
oracle's own elimination exactly, and the reduced signal must equal the
oracle's fold by that basis element for element (integers: bit-exact).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1607_01039_amd as F  # an import failure fails collection, never skips
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _native_library():
    """Every test here runs the HIP library: load it or fail."""
    assert torch.cuda.is_available()
    F._lib.lib()


TORCH = {np.int32: torch.int32, np.int64: torch.int64}


@pytest.fixture(scope="module")
def O():
    return oracle.get()


def _rows(n, m, seed):
    return synth.subspace_rows(n, m, seed) if m else np.zeros(0, dtype=np.uint64)


def _check_basis(rows, n, m, basis):
    if m == 0:
        assert basis.size == 0
        return
    want = oracle.gf2_canonical_rows(rows, n)
    assert [int(v) for v in basis] == want


# (n, m, seed): chunked partial sums (small m), m = n (a permutation), m = 0
# (the total), n - m < 3 (no unrolled steps), odd sizes, several tiles.
STORED = [(10, 4, 1), (12, 12, 2), (9, 0, 3), (13, 11, 4), (14, 13, 5), (16, 6, 6), (18, 9, 7),
          (20, 14, 8), (21, 17, 9), (22, 3, 10), (23, 20, 11), (24, 12, 12)]


@pytest.mark.parametrize("dt", [np.int32, np.int64], ids=["int32", "int64"])
@pytest.mark.parametrize("n,m,seed", STORED)
def test_fold_stored_matches_oracle(O, n, m, seed, dt):
    print(f"fold stored n={n} m={m} seed={seed} {dt.__name__}", flush=True)
    x = synth.ints(1 << n, 500 + seed, -(1 << 20), 1 << 20, dtype=dt)
    rows = _rows(n, m, seed)
    xd = torch.from_numpy(x).cuda()
    u, basis = F.fold_(xd, m, rows)
    torch.cuda.synchronize()
    _check_basis(rows, n, m, basis)
    if m == 0:
        want = np.array([x.astype(np.int64).sum()]).astype(dt)
    else:
        want = O.fold(x, basis, m)
    assert np.array_equal(u.cpu().numpy(), want)
    assert torch.equal(xd.cpu(), torch.from_numpy(x))  # the source is left alone


@pytest.mark.parametrize("dt", [np.int32, np.int64], ids=["int32", "int64"])
def test_fold_low_columns_dependent(O, dt):
    # Bits 0 and 1 are not both pivots: the reduction reads single entries.
    n, m = 16, 5
    rows = np.array([0b11, 0b1100, 1 << 7, (1 << 9) | 1, (1 << 15) | (1 << 4)], dtype=np.uint64)
    x = synth.ints(1 << n, 61, -1000, 1000, dtype=dt)
    u, basis = F.fold_(torch.from_numpy(x).cuda(), m, rows)
    _check_basis(rows, n, m, basis)
    assert np.array_equal(u.cpu().numpy(), O.fold(x, basis, m))


def test_fold_int32_wraps(O):
    n, m = 14, 3
    x = synth.ints(1 << n, 62, -(1 << 31), (1 << 31) - 1, dtype=np.int32)
    rows = _rows(n, m, 63)
    u, basis = F.fold_(torch.from_numpy(x).cuda(), m, rows)
    assert np.array_equal(u.cpu().numpy(), O.fold(x, basis, m))


def test_fold_reuses_output_and_smaller_second_call(O):
    out = torch.empty(1 << 10, dtype=torch.int64, device="cuda")
    for (n, m, seed) in ((20, 10, 70), (12, 10, 71)):
        x = synth.ints(1 << n, seed, -50, 50)
        u, basis = F.fold_(torch.from_numpy(x).cuda(), m, _rows(n, m, seed), out=out)
        assert u.data_ptr() == out.data_ptr()
        assert np.array_equal(u.cpu().numpy(), O.fold(x, basis, m))


GEN = [(8, 3, 1), (12, 12, 2), (14, 0, 3), (15, 13, 4), (16, 7, 5), (20, 12, 6), (22, 16, 7)]


@pytest.mark.parametrize("dt", [np.int32, np.int64], ids=["int32", "int64"])
@pytest.mark.parametrize("n,m,seed", GEN)
def test_fold_planted_matches_oracle(O, n, m, seed, dt):
    print(f"fold planted n={n} m={m} seed={seed} {dt.__name__}", flush=True)
    p = 0.45
    x, s, _ = synth.planted(n, 30 + seed, p, dtype=np.int64)
    mask, state, thr = synth.planted_params(n, 30 + seed, p)
    rows = _rows(n, m, seed)
    u, basis = F.fold_planted(n, m, rows, mask, state, thr, dtype=TORCH[dt])
    torch.cuda.synchronize()
    _check_basis(rows, n, m, basis)
    want = np.array([x.sum()]) if m == 0 else O.fold(x, basis, m)
    assert np.array_equal(u.cpu().numpy(), want.astype(dt))


@pytest.mark.parametrize("p", [0.0, 1.0])
def test_fold_planted_extreme_noise(O, p):
    # p = 0: no noise bit is ever set; p = 1: every one is (threshold 2^32).
    n, m = 14, 9
    x, s, errors = synth.planted(n, 13, p, dtype=np.int64)
    assert errors == (0 if p == 0.0 else 1 << n)
    mask, state, thr = synth.planted_params(n, 13, p)
    rows = _rows(n, m, 14)
    u, basis = F.fold_planted(n, m, rows, mask, state, thr)
    assert np.array_equal(u.cpu().numpy(), O.fold(x, basis, m))


def test_subspace_transform_hits(O):
    # Reduce, transform and threshold; the hits are the coefficients of the
    # full transform above T on the subspace, at full-space indices.
    n, m, p, seed = 20, 14, 0.45, 2
    x, s, errors = synth.planted(n, seed, p, dtype=np.int64)
    rows = _rows(n, m, 90)
    rows[0] = np.uint64(s)  # make the planted peak lie in the subspace
    assert oracle.gf2_rank(rows) == m
    W = O.wht_fig1(x)
    T = int(np.ceil(4.0 * 2 ** (n / 2)))
    u, basis = F.fold_(torch.from_numpy(x).cuda(), m, rows)
    hits = F.subspace_transform(u, basis, T, cap=1 << 12)
    ks = O.subspace_indices(basis, range(1 << m)).astype(np.int64)
    sub = W[ks]
    keep = np.abs(sub) > T
    want_k, want_v = ks[keep], sub[keep]
    order = np.argsort(want_k)
    got_k, got_v = hits.sorted()
    assert hits.count == keep.sum()
    assert np.array_equal(got_k, want_k[order]) and np.array_equal(got_v, want_v[order])
    assert s in set(got_k.tolist())
    assert W[s] == (1 << n) - 2 * errors
    # the transformed u holds the subspace coefficients in reduced order
    assert np.array_equal(u.cpu().numpy(), sub)


def test_subspace_hits_capacity(O):
    n, m = 12, 8
    x = synth.ints(1 << n, 91, -3, 3)
    rows = _rows(n, m, 92)
    u, basis = F.fold_(torch.from_numpy(x).cuda(), m, rows)
    hits = F.subspace_transform(u, basis, 0, cap=16)
    W = O.wht_fig1(x)
    ks = O.subspace_indices(basis, range(1 << m)).astype(np.int64)
    assert hits.count == int(np.count_nonzero(W[ks])) and hits.count > 16
    got_k, got_v = hits.sorted()
    assert got_k.size == 16 and np.array_equal(W[got_k], got_v)
    assert set(got_k.tolist()) <= set(ks.tolist())


def test_fold_planted_n40_to_2p30(O):
    # The on-the-fly workload at its benchmark size: 2^40 generated entries
    # reduced to 2^30, with the planted peak inside the subspace.  Checked on
    # sampled entries (each a direct sum over its 2^10 preimages), then the
    # transform's hit at the peak against a direct sum over u.
    n, m, p, seed = 40, 30, 0.45, 6
    mask, state, thr = synth.planted_params(n, seed, p)
    rows = synth.subspace_rows(n, m, 400)
    rows[0] = np.uint64(mask)
    assert oracle.gf2_rank(rows) == m
    print("fold planted n=40 m=30", flush=True)
    u, basis = F.fold_planted(n, m, rows, mask, state, thr)
    torch.cuda.synchronize()
    _check_basis(rows, n, m, basis)
    rng = np.random.default_rng(5)
    js = [0, (1 << m) - 1] + [int(v) for v in rng.integers(0, 1 << m, size=10)]
    got = u[torch.tensor(js, device="cuda")].cpu().numpy()
    for j, g in zip(js, got):
        pre = oracle.fold_preimage(basis, n, j)
        assert pre.size == 1 << (n - m)
        assert int(synth.planted_at(n, seed, p, pre).sum()) == int(g), j
    uh = u.cpu().numpy()
    print("transform 2^30 int64", flush=True)
    T = int(np.ceil(6 * 2 ** (n / 2)))
    hits = F.subspace_transform(u, basis, T, cap=1 << 12)
    got_k, got_v = hits.sorted()
    assert int(mask) in set(got_k.tolist())
    # the planted peak's reduced index: its bits at the basis pivots
    piv = [int(v) & -int(v) for v in basis]
    kp = sum(1 << t for t, pv in enumerate(piv) if int(mask) & pv)
    k_full = O.subspace_index(basis, kp)
    assert k_full == int(mask)
    k_of = {int(k): int(v) for k, v in zip(got_k, got_v)}
    direct = int(O.wht_def_at(uh, [kp])[0])
    assert k_of[k_full] == direct
    assert abs(direct) > (1 << n) // 20  # mean 2^n (1 - 2p) = 0.1 * 2^n


def test_fold_stored_n30_bench_size(O):
    # The stored workload of the benchmark (signs, seed 2, 2^30 int32 -> 2^24):
    # sampled entries against direct sums over their 64 preimages, and the total.
    n, m = 30, 24
    x = synth.signs(1 << n, 2)
    rows = synth.subspace_rows(n, m, 7)
    print("fold stored n=30 m=24", flush=True)
    xd = torch.from_numpy(x).cuda()
    u, basis = F.fold_(xd, m, rows)
    torch.cuda.synchronize()
    _check_basis(rows, n, m, basis)
    rng = np.random.default_rng(30)
    js = [0, 1, 2, 3, (1 << m) - 1] + [int(v) for v in rng.integers(0, 1 << m, size=60)]
    got = u[torch.tensor(js, device="cuda")].cpu().numpy()
    for j, g in zip(js, got):
        pre = oracle.fold_preimage(basis, n, j).astype(np.int64)
        assert pre.size == 1 << (n - m)
        assert int(x[pre].astype(np.int64).sum()) == int(g), j
    assert int(u.to(torch.int64).sum().item()) == int(x.astype(np.int64).sum())


def test_fold_planted_n44(O):
    # 2^44 generated entries (about 11 s) reduced to 2^30: each thread walks
    # 2^14 steps of h; sampled entries against direct sums over their 2^14
    # preimages, and the entry holding the planted peak's coefficient.
    n, m, p, seed = 44, 30, 0.45, 8
    mask, state, thr = synth.planted_params(n, seed, p)
    rows = synth.subspace_rows(n, m, 44)
    rows[0] = np.uint64(mask)
    assert oracle.gf2_rank(rows) == m
    print("fold planted n=44 m=30", flush=True)
    u, basis = F.fold_planted(n, m, rows, mask, state, thr, dtype=torch.int32)
    torch.cuda.synchronize()
    _check_basis(rows, n, m, basis)
    rng = np.random.default_rng(44)
    js = [0, (1 << m) - 1] + [int(v) for v in rng.integers(0, 1 << m, size=6)]
    got = u[torch.tensor(js, device="cuda")].cpu().numpy()
    for j, g in zip(js, got):
        pre = oracle.fold_preimage(basis, n, j)
        assert pre.size == 1 << (n - m)
        assert int(synth.planted_at(n, seed, p, pre).sum()) == int(g), j


def test_subspace_scan_union(O):
    # Section 5.1's scheme at a scale the oracle can check: 64 independent
    # reductions of 2^20 planted entries to 2^15 (1/32 of the coefficients
    # each, as in the paper's example).  The merged hits equal the oracle's
    # coefficients above T on the union of the 64 subspaces, and that union
    # covers close to 1 - (31/32)^64 = 87% of the spectrum.
    n, m, R, p, seed = 20, 15, 64, 0.45, 9
    mask, state, thr = synth.planted_params(n, seed, p)
    rows_list = [synth.subspace_rows(n, m, 700 + r) for r in range(R)]
    T = int(np.ceil(4 * 2 ** (n / 2)))
    hits, bases = F.subspace_scan((n, mask, state, thr), m, rows_list, T)
    x, s, _ = synth.planted(n, seed, p, dtype=np.int64)
    W = O.wht_fig1(x)
    covered = np.zeros(1 << n, dtype=bool)
    for b in bases:
        covered[O.subspace_indices(b, range(1 << m)).astype(np.int64)] = True
    want = {int(k): int(W[k]) for k in np.flatnonzero(covered & (np.abs(W) > T))}
    assert hits == want
    share = covered.mean()
    assert abs(share - (1 - (31 / 32) ** R)) < 0.02, share
