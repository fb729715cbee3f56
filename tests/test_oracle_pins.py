"""The CPU oracle against the paper's definitions and mathematical facts."""
import os
import tempfile

import numpy as np
import pytest

import oracle
import synth
from oracle_pins import ALL_PINS


@pytest.mark.parametrize("pin", ALL_PINS, ids=lambda f: f.__name__)
def test_pin(O, pin):
    assert O.mutant == 0
    pin(O)


# Each id plants one plausible mistake in a copy of the oracle (see the
# ORACLE_MUTANT branches of wht_oracle.c): 1 butterfly signs swapped,
# 2 last stage dropped, 3 "-b" term dropped, 4 bit-reversed output order,
# 5 definition sign flipped, 6 OR instead of AND in <i,j>, 7 hit index off by
# one, 8 ">=" instead of ">", 9 sign of the coefficient ignored in |y|,
# 10 scale 2^-n instead of 2^-n/2, 11 Fig. 2 workload starts that ignore the
# gap at bit k, 12 rows of the reduction map applied in reverse order, 13 OR
# instead of XOR when mapping a reduced index back to the full space, 14 a
# square factor 2^2 counted once in the prime-factor counts, 15 the last prime
# factor above the square root dropped by trial division, 16 the signs of the
# input-side weights of the randomized transform check swapped, 17 a negative
# entry reduced mod 2^61 - 1 as if unsigned, 18 the check's random point
# ignored (every weight collapses onto index 0), 19 the last entry of each
# thread's part left out of the Parseval sums.
MUTANTS = list(range(1, 20))


@pytest.mark.parametrize("mutant", MUTANTS)
def test_pins_catch_planted_mistake(mutant):
    with tempfile.TemporaryDirectory() as d:
        path = oracle.build(os.path.join(d, f"liboracle_m{mutant}.so"), mutant=mutant)
        M = oracle.Oracle(path)
        assert M.mutant == mutant
        failed = []
        for pin in ALL_PINS:
            try:
                pin(M)
            except AssertionError:
                failed.append(pin.__name__)
        assert failed, f"mutant {mutant} passed every pin"


def test_splitmix64_published_outputs():
    # First three outputs of SplitMix64 (Steele, Lea & Flood 2014) from state 0,
    # as produced by the published reference generator.
    golden = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_state0.txt")
    want = [int(l.split()[0], 16) for l in open(golden) if l.strip() and not l.startswith("#")]
    got = [int(v) for v in synth.splitmix64(0, 0, len(want))]
    assert got == want


@pytest.mark.parametrize("n,seed,p,start", [(0, 1, 0.45, 0), (7, 2, 0.45, 0),
                                            (13, 3, 0.48, 0), (20, 2, 0.45, 12345)])
def test_synth_c_matches_definition(n, seed, p, start):
    N = 1 << n
    cnt = min(N - start, 1 << 15)
    for dt in (np.int32, np.int64):
        a = synth.planted(n, seed, p, dtype=dt, start=start, count=cnt)
        b = synth.planted_ref(n, seed, p, dtype=dt, start=start, count=cnt)
        assert np.array_equal(a[0], b[0]) and a[1] == b[1] and a[2] == b[2]
    assert np.array_equal(synth.signs(1000, seed), synth.signs_ref(1000, seed))
    raw = synth.raw64(1000, seed)
    assert np.array_equal(raw.view(np.uint64), synth.splitmix64(synth.stream_state(seed, 3), 0, 1000))


def test_planted_noise_statistics(O):
    # Section 2: noise coefficients are approximately N(0, 2^n sigma^2) with
    # sigma^2 = 1 - mu^2, mu = 1 - 2p (a sanity check, not a pin).
    n, p = 18, 0.45
    x, s, _ = synth.planted(n, 2, p)
    y = O.wht_fig1(x).astype(np.float64)
    y[s] = 0
    var = np.mean(y * y)
    want = (1 << n) * (1 - (1 - 2 * p) ** 2)
    assert abs(var / want - 1) < 0.02
    assert abs(np.mean(y)) < 4 * np.sqrt(want / (1 << n))
