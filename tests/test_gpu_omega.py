"""Prime-factor counts (the workload announced in section 4.3) on the GPU
against the oracle, and their transform on the int64 path."""
import numpy as np
import pytest
import torch

import oracle
import paper_1607_01039_amd as F  # an import failure fails collection, never skips

pytestmark = pytest.mark.gpu

@pytest.fixture(scope="module", autouse=True)
def _native_library():
    """Every test here runs the HIP library: load it or fail."""
    assert torch.cuda.is_available()
    F._lib.lib()


@pytest.fixture(scope="module")
def O():
    return oracle.get()


# one partial segment (n < 15), exactly one, several, and many per workgroup
@pytest.mark.parametrize("n", [0, 1, 2, 3, 5, 9, 14, 15, 16, 19, 22, 24])
@pytest.mark.parametrize("dt", [torch.int32, torch.int64], ids=["int32", "int64"])
def test_prime_omega_matches_oracle(O, n, dt):
    print(f"prime omega n={n} {dt}", flush=True)
    got = F.prime_omega(n, dtype=dt).cpu().numpy()
    assert np.array_equal(got, O.prime_omega(1 << n).astype(got.dtype))


def _legendre(N):
    """sum over prime powers p^k <= N of floor(N / p^k) (primes by a boolean sieve)."""
    ok = np.ones(N + 1, dtype=bool)
    ok[:2] = False
    for p in range(2, int(N ** 0.5) + 1):
        if ok[p]:
            ok[p * p::p] = False
    q = np.flatnonzero(ok).astype(np.int64)
    del ok
    ps, tot = q.copy(), 0
    while q.size:
        tot += int((N // q).sum())
        keep = q <= N // ps
        q, ps = q[keep] * ps[keep], ps[keep]
    return tot


def test_prime_omega_transform_parity(O):
    # The whole pipeline at n = 22 against the oracle bit for bit.
    n = 22
    x = F.prime_omega(n)
    hits = F.fwht_int_(x, threshold=(1 << n) // 16, cap=1 << 12)
    W = O.wht_fig1(O.prime_omega(1 << n).astype(np.int64))
    assert np.array_equal(x.cpu().numpy(), W)
    k, v = hits.sorted()
    want = np.flatnonzero(np.abs(W) > (1 << n) // 16)
    assert np.array_equal(k, want) and np.array_equal(v, W[want])


@pytest.mark.parametrize("n", [28, 30])
def test_prime_omega_large(O, n):
    # At full size: sampled entries (including the last ones and powers of
    # primes) against trial division, and the total against Legendre's
    # formula, which is also the transform's coefficient at k = 0.
    print(f"prime omega n={n}", flush=True)
    x = F.prime_omega(n)
    rng = np.random.default_rng(n)
    ks = [(1 << n) - 1, (1 << n) - 2, 1 << (n - 1), 3 ** 18, 65521 * 65519 if n >= 32 else 32749 * 32719,
          2 * 32749 * 32719 if n >= 31 else 32749 * 16381] + [int(v) for v in rng.integers(0, 1 << n, 2000)]
    ks = [k for k in ks if k < (1 << n)]
    got = x[torch.tensor(ks, device="cuda")].cpu().numpy()
    assert np.array_equal(got, O.prime_omega_at(ks))
    total = _legendre((1 << n) - 1)
    assert int(x.sum().item()) == total
    print("transform", flush=True)
    hits = F.fwht_int_(x, threshold=(1 << n) // 8, cap=1 << 10)
    k, v = hits.sorted()
    assert k[0] == 0 and v[0] == total


def test_prime_omega_n30_every_entry(O):
    # The benchmark size: all 2^30 entries (int64 on the device) against the
    # oracle's sieve, chunk by chunk.
    n, C = 30, 1 << 26
    print("prime omega n=30 (every entry)", flush=True)
    x = F.prime_omega(n)
    ref = O.prime_omega(1 << n)
    for c0 in range(0, 1 << n, C):
        got = x[c0:c0 + C].cpu().numpy()
        assert np.array_equal(got, ref[c0:c0 + C].astype(np.int64)), c0
    del x
    torch.cuda.empty_cache()


def test_prime_omega_n32(O):
    # The largest size (indices and prime powers up to 2^32 - 1): sampled
    # entries, including the top of the range and squares of the largest
    # sieving primes, against trial division; int32 output equals int64.
    n = 32
    x = F.prime_omega(n, dtype=torch.int32)
    rng = np.random.default_rng(32)
    ks = [(1 << 32) - 1, (1 << 32) - 2, (1 << 32) - 5, 65521 * 65519, 65521 * 65521 if 65521 ** 2 < 1 << 32 else 3,
          3 ** 20, 2 ** 31, 65537 * 65519, 4294967291] + [int(v) for v in rng.integers(0, 1 << 32, 3000, dtype=np.uint64)]
    got = x[torch.tensor(np.array(ks, dtype=np.int64), device="cuda")].cpu().numpy()
    assert np.array_equal(got.astype(np.int64), O.prime_omega_at(ks))
    del x
    torch.cuda.empty_cache()
