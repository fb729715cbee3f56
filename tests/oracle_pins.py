"""Pins for the CPU oracle: facts fixed by the paper and by mathematics.

Each ``pin_*`` takes an ``oracle.Oracle`` and raises AssertionError when the
oracle disagrees with something other than itself:

* the Sylvester Hadamard matrix, built two independent ways (scipy's
  ``hadamard`` and Kronecker powers of [[1, 1], [1, -1]]), which in natural
  order is the matrix of Eq. 2 (section 2);
* closed forms: e_0 -> all ones, a constant c -> c 2^n delta_0, the Walsh
  function chi_s -> 2^n delta_s, the planted peak W(s) = 2^n - 2 #errors;
* identities: the involution H(Hx) = 2^n x, Parseval sum W^2 = 2^n sum x^2,
  linearity, and reduction mod 2^32 of an exact 64-bit result;
* the three algorithms of the paper (Fig. 1, Fig. 2, Fig. 3), which must
  agree bit for bit on integers;
* the threshold pass of the problem statement (strict |y_k| > T, ascending
  k, true count beyond the capacity);
* the orthonormal scale 2^(-n/2) and the gradient of a weighted square loss,
  checked by central finite differences (exact for a quadratic up to
  rounding);
* the checks used where no oracle copy of a transform fits: the randomized
  identity sum_k W_k w_k = sum_i x_i (H w)_i for Kronecker-product weights
  (mod 2^61 - 1) and Parseval's identity mod 2^64 and mod 2^61 - 1, against
  the Fig. 1 transform, corrupted transforms and sums written out over
  Python integers.

The mutation test runs every pin against builds of the oracle with a planted
mistake and requires each such build to fail at least one pin.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

import oracle
import synth


def _sylvester_kron(n: int) -> np.ndarray:
    H = np.ones((1, 1), dtype=np.int64)
    H2 = np.array([[1, 1], [1, -1]], dtype=np.int64)
    for _ in range(n):
        H = np.kron(H2, H)
    return H


def pin_def_vs_sylvester(O):
    for n in range(0, 10):
        x = synth.ints(1 << n, 100 + n, -1000, 1000)
        H = scipy.linalg.hadamard(1 << n).astype(np.int64)
        assert np.array_equal(O.wht_def(x), H @ x), n
        assert np.array_equal(_sylvester_kron(n) @ x, H @ x), n
        xf = synth.normal(1 << n, 200 + n).astype(np.float64)
        assert np.allclose(O.wht_def(xf), H.astype(np.float64) @ xf, rtol=0, atol=1e-9), n


def pin_def_at_vs_sylvester(O):
    for n in (3, 7, 10):
        H = scipy.linalg.hadamard(1 << n).astype(np.int64)
        x32 = synth.ints(1 << n, 7 + n, -(1 << 20), 1 << 20, dtype=np.int32)
        x64 = synth.ints(1 << n, 9 + n, -(1 << 40), 1 << 40, dtype=np.int64)
        ks = [0, 1, (1 << n) - 1, (1 << n) // 3]
        assert np.array_equal(O.wht_def_at(x32, ks), (H @ x32.astype(np.int64))[ks])
        assert np.array_equal(O.wht_def_at(x64, ks), (H @ x64)[ks])


def pin_fig1_vs_sylvester(O):
    for n in range(0, 11):
        H = scipy.linalg.hadamard(1 << n).astype(np.int64)
        x = synth.ints(1 << n, 300 + n, -1000, 1000)
        ref = H @ x
        assert np.array_equal(O.wht_fig1(x.astype(np.int32)), ref.astype(np.int32)), n
        assert np.array_equal(O.wht_fig1(x), ref), n
        xf = synth.normal(1 << n, 400 + n)
        assert np.allclose(O.wht_fig1(xf), H @ xf.astype(np.float64), rtol=0, atol=1e-9), n


def pin_fig1_vs_def(O):
    for n in (11, 12):
        x = synth.ints(1 << n, 500 + n, -(1 << 20), 1 << 20)
        assert np.array_equal(O.wht_fig1(x), O.wht_def(x)), n


def pin_closed_forms(O):
    for n in (1, 5, 13, 18):
        N = 1 << n
        d = np.zeros(N, dtype=np.int32)
        d[0] = 1
        assert np.array_equal(O.wht_fig1(d), np.ones(N, dtype=np.int32)), n
        c = np.full(N, -3, dtype=np.int64)
        want = np.zeros(N, dtype=np.int64)
        want[0] = -3 * N
        assert np.array_equal(O.wht_fig1(c), want), n
        # Walsh function chi_s: the planted signal with no noise (p = 0).
        chi, s, err = synth.planted(n, 11 + n, 0.0, dtype=np.int32)
        assert err == 0
        want = np.zeros(N, dtype=np.int32)
        want[s] = N
        assert np.array_equal(O.wht_fig1(chi), want), n


def pin_closed_forms_def(O):
    n = 8
    N = 1 << n
    d = np.zeros(N, dtype=np.int64)
    d[0] = 1
    assert np.array_equal(O.wht_def(d), np.ones(N, dtype=np.int64))
    chi, s, _ = synth.planted(n, 5, 0.0, dtype=np.int64)
    want = np.zeros(N, dtype=np.int64)
    want[s] = N
    assert np.array_equal(O.wht_def(chi), want)
    assert O.wht_def_at(chi, [s])[0] == N


def pin_involution_parseval(O):
    for n in (4, 12, 16):
        N = 1 << n
        x = synth.ints(N, 600 + n, -100, 100)
        y = O.wht_fig1(x)
        assert np.array_equal(O.wht_fig1(y), N * x), n
        assert int(np.sum(y * y)) == N * int(np.sum(x * x)), n


def pin_linearity_and_wrap(O):
    n = 12
    N = 1 << n
    a = synth.ints(N, 1, -(1 << 30), 1 << 30)
    b = synth.ints(N, 2, -(1 << 30), 1 << 30)
    wa, wb = O.wht_fig1(a), O.wht_fig1(b)
    assert np.array_equal(O.wht_fig1(3 * a - 5 * b), 3 * wa - 5 * wb)
    # int32 results are the exact 64-bit results reduced mod 2^32.
    a32 = a.astype(np.int32)
    exact = O.wht_fig1(a32.astype(np.int64))
    assert np.array_equal(O.wht_fig1(a32), exact.astype(np.int32))
    assert np.any(np.abs(exact) > (1 << 31))  # the case really wraps


def pin_planted_peak(O):
    for n, p, seed in ((16, 0.45, 2), (20, 0.45, 3), (18, 0.48, 4)):
        x, s, err = synth.planted(n, seed, p, dtype=np.int32)
        y = O.wht_fig1(x)
        assert int(y[s]) == (1 << n) - 2 * err, n
        assert int(np.argmax(np.abs(y.astype(np.int64)))) == s, n
        assert int(O.wht_def_at(x, [s])[0]) == (1 << n) - 2 * err, n


def pin_fig2_fig3(O):
    for n, qs in ((3, (0, 1, 2)), (10, (0, 1, 2, 3)), (16, (1, 2, 4))):
        x32 = synth.signs(1 << n, 20 + n)
        x64 = synth.ints(1 << n, 30 + n, -(1 << 40), 1 << 40)
        r32, r64 = O.wht_fig1(x32), O.wht_fig1(x64)
        for q in qs:
            assert np.array_equal(O.wht_fig2(x32, q), r32), (n, q)
            assert np.array_equal(O.wht_fig2(x64, q), r64), (n, q)
        for B in range(0, n + 1, 3):
            assert np.array_equal(O.wht_fig3(x64, B), r64), (n, B)


def pin_threshold(O):
    y = np.array([5, -7, 0, 7, -2147483648, 2147483647, 6, -6], dtype=np.int32)
    idx, val, cnt = O.threshold(y, 6)
    assert cnt == 4 and list(idx) == [1, 3, 4, 5] and list(val) == [-7, 7, -2147483648, 2147483647]
    idx, val, cnt = O.threshold(y, 6, cap=2)
    assert cnt == 4 and list(idx) == [1, 3]
    idx, val, cnt = O.threshold(y, -1)
    assert cnt == 8 and list(idx) == list(range(8))
    idx, val, cnt = O.threshold(y, 2147483647)
    assert cnt == 1 and list(idx) == [4]
    y64 = np.array([-(1 << 62), 1 << 40, -(1 << 63), 3], dtype=np.int64)
    idx, val, cnt = O.threshold(y64, 1 << 40)
    assert cnt == 2 and list(idx) == [0, 2]
    yf = np.array([0.5, -1.5, 1.0, -1.0, 2.0], dtype=np.float64)
    idx, val, cnt = O.threshold(yf, 1.0)
    assert cnt == 2 and list(idx) == [1, 4] and list(val) == [-1.5, 2.0]
    # against a numpy scan of a transformed planted signal
    x, s, _ = synth.planted(14, 9, 0.3)
    w = O.wht_fig1(x)
    T = 6 * (1 << 7)
    idx, val, cnt = O.threshold(w, T)
    want = np.nonzero(np.abs(w.astype(np.int64)) > T)[0]
    assert cnt == len(want) and np.array_equal(idx, want) and np.array_equal(val, w[want])
    assert s in set(idx.tolist())


def pin_orthonormal(O):
    for n in (0, 1, 5, 10):
        N = 1 << n
        assert abs(O.orthonormal_scale(n) ** 2 * N - 1.0) < 1e-15
        x = synth.normal((3, N), 40 + n).astype(np.float64)
        y = O.wht_batch(x, n, True)
        assert np.allclose(O.wht_batch(y, n, True), x, rtol=0, atol=1e-12)
        assert np.allclose((y * y).sum(1), (x * x).sum(1), rtol=1e-13)
        H = scipy.linalg.hadamard(N).astype(np.float64)
        assert np.allclose(y, x @ H / np.sqrt(N), rtol=0, atol=1e-12)


def pin_ragged(O):
    lg, off, tot = synth.ragged(9, 0, 7, 3)
    x = synth.normal(tot, 5)
    y = O.wht_ragged(x, off, lg, True)
    for t in range(9):
        N = 1 << int(lg[t])
        seg = x[off[t]:off[t] + N].astype(np.float64)
        H = scipy.linalg.hadamard(N).astype(np.float64)
        assert np.allclose(y[off[t]:off[t] + N], H @ seg / np.sqrt(N), rtol=0, atol=1e-12)


def pin_gradient(O):
    n, B = 5, 2
    N = 1 << n
    x = synth.normal((B, N), 7).astype(np.float64)
    w = synth.uniform((B, N), 8).astype(np.float64)
    g = O.grad_weighted_square(x, w, n)
    H = scipy.linalg.hadamard(N).astype(np.float64) / np.sqrt(N)

    def loss(z):
        return float(np.sum(w * (z @ H) ** 2))

    eps = 1e-3
    fd = np.zeros_like(x)
    for b in range(B):
        for i in range(N):
            e = np.zeros_like(x)
            e[b, i] = eps
            fd[b, i] = (loss(x + e) - loss(x - e)) / (2 * eps)
    assert np.allclose(g, fd, rtol=1e-8, atol=1e-8)


def pin_norms(O):
    lg, off, tot = synth.ragged(5, 1, 6, 4)
    x = synth.normal(tot, 1)
    y = synth.normal(tot, 2)
    r = synth.normal(tot, 3).astype(np.float64)
    sx, sy, se = O.norms(x, y, r, off, lg)
    for t in range(5):
        sl = slice(off[t], off[t] + (1 << int(lg[t])))
        xd, yd = x[sl].astype(np.float64), y[sl].astype(np.float64)
        assert np.isclose(sx[t], np.dot(xd, xd), rtol=1e-14)
        assert np.isclose(sy[t], np.dot(yd, yd), rtol=1e-14)
        assert np.isclose(se[t], np.dot(yd - r[sl], yd - r[sl]), rtol=1e-14)


# ---- section 5.1: linear space reduction ------------------------------------

def _map_numpy(rows, n):
    """A i for every i in [0, 2^n), by brute force (bit t = parity(rows[t] & i))."""
    i = np.arange(1 << n, dtype=np.uint64)
    j = np.zeros(1 << n, dtype=np.uint64)
    for t, r in enumerate(rows):
        j |= (np.bitwise_count(i & np.uint64(int(r))) & np.uint8(1)).astype(np.uint64) << np.uint64(t)
    return j


def pin_fold_vs_sylvester(O):
    # The 2^m-point transform of the reduced signal u equals the full
    # transform on the subspace {A^T k'}: both sides by Hadamard matrices.
    for (n, m, seed) in ((6, 3, 1), (8, 5, 2), (9, 9, 3), (7, 1, 4), (10, 6, 5)):
        rows = synth.subspace_rows(n, m, seed)
        x = synth.ints(1 << n, 40 + seed, -50, 50)
        W = scipy.linalg.hadamard(1 << n, dtype=np.int64) @ x
        u = O.fold(x, rows, m)
        Wu = scipy.linalg.hadamard(1 << m, dtype=np.int64) @ u
        ks = O.subspace_indices(rows, range(1 << m)).astype(np.int64)
        assert np.array_equal(Wu, W[ks]), (n, m)
        # the subspace has 2^m distinct members
        assert len(set(ks.tolist())) == 1 << m
        # int32 folds wrap like the int64 ones
        u32 = O.fold(x.astype(np.int32), rows, m)
        assert np.array_equal(u32, u.astype(np.int32))


def pin_fold_special_maps(O):
    # A = [I_m | 0] sums the 2^(n-m) blocks of 2^m consecutive entries;
    # an invertible A (m = n) permutes x; every fold preserves the total
    # (W(0) = sum x_i); the preimage of each j has 2^(n-m) members.
    n, m = 9, 4
    x = synth.ints(1 << n, 77, -1000, 1000)
    u = O.fold(x, [1 << t for t in range(m)], m)
    assert np.array_equal(u, x.reshape(-1, 1 << m).sum(axis=0))
    rows = synth.subspace_rows(n, n, 8)
    up = O.fold(x, rows, n)
    assert np.array_equal(np.sort(up), np.sort(x))
    j = _map_numpy(rows, n)
    assert np.array_equal(up[j.astype(np.int64)], x)
    rows = synth.subspace_rows(n, m, 9)
    u = O.fold(x, rows, m)
    assert int(u.sum()) == int(x.sum())
    jm = _map_numpy(rows, n)
    assert np.array_equal(np.bincount(jm.astype(np.int64), minlength=1 << m),
                          np.full(1 << m, 1 << (n - m)))


def pin_fold_planted_peak(O):
    # Noise-free planted signal (p = 0) is the Walsh function chi_s: the
    # reduced transform is 2^n at the k' with A^T k' = s when s lies in the
    # subspace (rank test), and zero everywhere else.
    n, m = 12, 5
    x, s, err = synth.planted(n, 11, 0.0, np.int64)
    assert err == 0
    found = 0
    for seed in range(40):
        rows = synth.subspace_rows(n, m, 100 + seed)
        if seed == 0:  # force one subspace through s
            rows = np.array([s] + [int(v) for v in rows[1:]], dtype=np.uint64)
            if oracle.gf2_rank(rows) < m:
                continue
        Wu = O.wht_fig1(O.fold(x, rows, m))
        inside = oracle.gf2_rank(list(rows) + [s]) == m
        nz = np.flatnonzero(Wu)
        if inside:
            found += 1
            assert nz.size == 1 and Wu[nz[0]] == 1 << n
            assert O.subspace_index(rows, int(nz[0])) == s
        else:
            assert nz.size == 0
    assert found >= 1


def pin_canonical_rows_and_preimage(O):
    # The reduced echelon basis spans the same space (brute-force spans) and
    # has unit pivot columns; fold_preimage agrees with a brute-force scan.
    for (n, m, seed) in ((8, 4, 1), (7, 7, 2), (9, 3, 3), (6, 1, 4)):
        rows = synth.subspace_rows(n, m, 200 + seed)
        can = oracle.gf2_canonical_rows(rows, n)
        assert can is not None and len(can) == m

        def span(rs):
            out = {0}
            for r in rs:
                out |= {v ^ int(r) for v in out}
            return out
        assert span(rows) == span(can)
        piv = [v & -v for v in can]
        assert piv == sorted(piv) and len(set(piv)) == m
        for t, v in enumerate(can):
            for q, p in enumerate(piv):
                assert bool(v & p) == (q == t)
        jm = _map_numpy(rows, n)
        for j in (0, 1, (1 << m) - 1, (5 * seed) % (1 << m)):
            want = np.flatnonzero(jm == j).astype(np.uint64)
            assert np.array_equal(oracle.fold_preimage(rows, n, j), want)
    dep = [3, 5, 6]  # 3 ^ 5 = 6
    assert oracle.gf2_canonical_rows(dep, 4) is None and oracle.gf2_rank(dep) == 2


def pin_subspace_coverage_example():
    # Section 5.1's worked example: each reduction keeps 1/32 of the
    # coefficients and 64 independent reductions cover about 87% of them.
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "subspace_coverage.txt")
    kv = dict(l.split()[:2] for l in open(path) if l.strip() and not l.startswith("#"))
    from fractions import Fraction
    frac = float(Fraction(kv["fraction_per_reduction"]))
    R, want = int(kv["reductions"]), float(kv["covered"])
    assert round(1 - (1 - frac) ** R, 2) == want


def pin_subspace_coverage(O):
    # The same example scaled down to n = 10, m = 5 (fraction 1/32): the
    # share of the 2^n - 1 nonzero coefficients that 64 random reductions
    # reach is close to 1 - (1 - (2^m - 1)/(2^n - 1))^64.
    pin_subspace_coverage_example()
    n, m, R = 10, 5, 64
    seen = np.zeros(1 << n, dtype=bool)
    for r in range(R):
        rows = synth.subspace_rows(n, m, 1000 + r)
        seen[O.subspace_indices(rows, range(1 << m)).astype(np.int64)] = True
    got = np.count_nonzero(seen[1:]) / ((1 << n) - 1)
    p = ((1 << m) - 1) / ((1 << n) - 1)
    assert abs(got - (1 - (1 - p) ** R)) < 0.03, got


# ---- prime-factor counts (section 4.3's announced workload) ----------------

def _primes_upto(n):
    """Sieve of Eratosthenes (boolean numpy), independent of the oracle."""
    ok = np.ones(n + 1, dtype=bool)
    ok[:2] = False
    for p in range(2, int(n ** 0.5) + 1):
        if ok[p]:
            ok[p * p::p] = False
    return np.flatnonzero(ok)


def pin_omega_definition(O):
    # Omega of 0 .. 20 written out from the factorisations (0 and 1 have none).
    want = [0, 0, 1, 1, 2, 1, 2, 1, 3, 2, 2, 1, 3, 1, 2, 2, 4, 1, 3, 1, 3]
    assert O.prime_omega(21).tolist() == want
    assert O.prime_omega_at(range(21)).tolist() == want
    om = O.prime_omega(1 << 16)
    ps = _primes_upto((1 << 16) - 1)
    assert np.all(om[ps] == 1)
    for p in (2, 3, 5, 7, 251):
        k = 1
        while p ** k < (1 << 16):
            assert om[p ** k] == k
            k += 1
    assert om.sum() == int(O.prime_omega_at(range(1 << 16)).sum())


def pin_omega_additive_and_legendre(O):
    # Omega is completely additive, Omega(ab) = Omega(a) + Omega(b), and by
    # Legendre's formula sum_{i <= N} Omega(i) = sum over prime powers p^k <= N
    # of floor(N / p^k).
    n = 20
    N = (1 << n) - 1
    om = O.prime_omega(1 << n)
    rng = np.random.default_rng(3)
    a = rng.integers(1, 1 << 10, size=2000)
    b = rng.integers(1, 1 << 10, size=2000)
    assert np.array_equal(om[a * b], om[a] + om[b])
    tot = 0
    for p in _primes_upto(N).tolist():
        q = p
        while q <= N:
            tot += N // q
            q *= p
    assert int(om.astype(np.int64).sum()) == tot
    # trial division on large numbers: products of known primes
    ps = _primes_upto(40000)
    for (x, k) in ((1 << 30, 30), (3 ** 18, 18), (int(ps[-1]) * int(ps[-2]), 2),
                   (int(ps[-1]) * int(ps[100]) * 4, 4), (int(ps[-1]) ** 2, 2), (int(ps[-1]), 1)):
        assert O.prime_omega_at([x])[0] == k, x


def pin_omega_threads(O):
    # The sieve splits the index range over threads: the result must not
    # depend on how (ragged parts, more threads than small primes), and a
    # range that ends just past a square of a prime keeps that square's count.
    for count in (2, 3, 50, 10007, 1 << 17):
        ref = O.prime_omega(count, threads=1)
        for th in (2, 3, 7, 16):
            assert np.array_equal(O.prime_omega(count, threads=th), ref), (count, th)
    assert O.prime_omega(122, threads=5)[121] == 2 and O.prime_omega(10202, threads=9)[10201] == 2


# ---- checks for transforms too large to keep an oracle copy of -------------

_KF_P = (1 << 61) - 1


def _kf_brute(y, n, t, side):
    """sum_k y_k w_side(k) mod P written out over Python integers."""
    acc = 0
    for k in range(1 << n):
        w = 1
        for j in range(n):
            bit = (k >> j) & 1
            if side == 0:
                w = w * (t[j] if bit else 1) % _KF_P
            else:
                w = w * ((1 - t[j]) if bit else (1 + t[j])) % _KF_P
        acc = (acc + int(y[k]) * w) % _KF_P
    return acc


def pin_kf_identity(O):
    # sum_k W_k prod_j t_j^(k_j) = sum_i x_i prod_j (1 + (-1)^(i_j) t_j) (mod P)
    # holds for the transform (Fig. 1) and for no plausible corruption of it.
    rng = np.random.default_rng(17)
    for n in (0, 1, 5, 12, 18):
        N = 1 << n
        x = synth.ints(N, 700 + n, -(1 << 40), 1 << 40)
        W = O.wht_fig1(x)
        for trial in range(2):
            t = [int(v) for v in rng.integers(0, _KF_P, size=max(n, 1), dtype=np.uint64)]
            lhs, rhs = O.kf_sum(W, n, t, 0), O.kf_sum(x, n, t, 1)
            assert lhs == rhs, (n, trial)
            if n >= 1:
                bad = W.copy(); bad[N // 3] += 1
                assert O.kf_sum(bad, n, t, 0) != rhs, n
                bad = W.copy(); bad[[0, N - 1]] = bad[[N - 1, 0]]
                assert W[0] == W[N - 1] or O.kf_sum(bad, n, t, 0) != rhs, n
                assert O.kf_sum(-W, n, t, 0) != rhs, n
            if n >= 2:
                rev = np.array([int(format(k, f"0{n}b")[::-1], 2) for k in range(N)])
                assert O.kf_sum(W[rev], n, t, 0) != rhs, n
    # int32 data, and sums taken chunk by chunk at arbitrary boundaries
    n = 16
    x = synth.signs(1 << n, 71)
    W = O.wht_fig1(x)
    t = [int(v) for v in rng.integers(0, _KF_P, size=n, dtype=np.uint64)]
    whole = O.kf_sum(W, n, t, 0)
    cuts = [0, 1, 4097, 30000, 1 << n]
    parts = sum(O.kf_sum(W[a:b], n, t, 0, start=a) for a, b in zip(cuts[:-1], cuts[1:])) % _KF_P
    assert parts == whole == O.kf_sum(x, n, t, 1)
    assert O.kf_sum(W, n, t, 0, threads=1) == O.kf_sum(W, n, t, 0, threads=13) == whole


def pin_kf_brute_force(O):
    # The C sums against the weights written out over Python integers
    # (extreme residues of t included), on transformed and untransformed data.
    rng = np.random.default_rng(5)
    for n in (1, 3, 6):
        x = synth.ints(1 << n, 800 + n, -(1 << 62), 1 << 62)
        x[0] = np.iinfo(np.int64).min
        for t in ([0] * n, [_KF_P - 1] * n, [int(v) for v in rng.integers(0, _KF_P, size=n, dtype=np.uint64)]):
            for side in (0, 1):
                assert O.kf_sum(x, n, t, side) == _kf_brute(x, n, t, side), (n, side)


def pin_parseval_mod(O):
    # Parseval (section 2): sum_k W_k^2 = 2^n sum_i x_i^2, exact in Python
    # integers and then reduced mod 2^64 and mod P; a one-unit error in any
    # coefficient changes the sum by 2 W_k + 1, an odd number.
    for n in (0, 3, 12, 17):
        N = 1 << n
        x = synth.ints(N, 900 + n, -(1 << 20), 1 << 20)
        W = O.wht_fig1(x)
        exact = sum(int(v) * int(v) for v in x.tolist()) * N
        assert O.sumsq(W) == exact % (1 << 64), n
        assert O.sumsq(W, mod_p=True) == exact % _KF_P, n
        assert O.sumsq(x.astype(np.int32), mod_p=True) == (exact // N) % _KF_P, n
        bad = W.copy(); bad[N - 1] += 1
        assert O.sumsq(bad) != exact % (1 << 64), n
    big = np.array([np.iinfo(np.int64).min, -3, (1 << 40) + 7], dtype=np.int64)
    ex = sum(int(v) * int(v) for v in big.tolist())
    assert O.sumsq(big) == ex % (1 << 64) and O.sumsq(big, mod_p=True) == ex % _KF_P


ALL_PINS = [v for k, v in sorted(globals().items()) if k.startswith("pin_") and k != "pin_subspace_coverage_example"]
