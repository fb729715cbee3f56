"""GPU parity of the integer transform and the threshold pass against the oracle.

Integer results must be bit-exact (wrap-around mod 2^32 / 2^64).  Hit lists
are compared as sets of (k, W_k) with the true count.
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


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _run_int(F, x, **kw):
    t = _dev(x)
    hits = F.fwht_int_(t, **kw)
    return t.cpu().numpy(), hits


@pytest.mark.parametrize("n", list(range(0, 23)))
def test_int32_every_n(F, O, n):
    x = synth.ints(1 << n, 1000 + n, -(1 << 20), 1 << 20, dtype=np.int32)
    y, _ = _run_int(F, x)
    assert np.array_equal(y, O.wht_fig1(x))


@pytest.mark.parametrize("n", [0, 1, 2, 3, 5, 8, 11, 12, 13, 14, 17, 20, 21])
def test_int64_every_n(F, O, n):
    x = synth.ints(1 << n, 2000 + n, -(1 << 40), 1 << 40, dtype=np.int64)
    y, _ = _run_int(F, x)
    assert np.array_equal(y, O.wht_fig1(x))


@pytest.mark.parametrize("n", [1, 4, 9, 12])
def test_int_matches_definition(F, O, n):
    x = synth.ints(1 << n, 3000 + n, -50, 50, dtype=np.int32)
    y, _ = _run_int(F, x)
    assert np.array_equal(y.astype(np.int64), O.wht_def(x.astype(np.int64)))


def test_int32_wraps_like_oracle(F, O):
    n = 14
    x = synth.ints(1 << n, 7, -(1 << 31), (1 << 31) - 1, dtype=np.int32)
    y, _ = _run_int(F, x)
    assert np.array_equal(y, O.wht_fig1(x))


SCHEDULES_I32 = {
    20: ["C12,S12c5:7,S14c6:1", "C14:6,S14c6:8,S13c6:6", "C15:15,S12c5:5", "C13:9,S15c6:9,S13c5:2",
         "C12:6,S12c5:7,S12c5:7"],
    26: ["C12,S14c6,S14c6:6", "C15,S15c6:9,S12c5:2", "C14,S13c6:6,S13c6:6"],
}
SCHEDULES_I64 = {
    20: ["C11,S12c4:8,S13c5:1", "C14:6,S14c5,S12c4:5", "C13,S13c6:7"],
}


def _variant_cases(dtype):
    """(variant, n, spec): every compiled variant once as the only pass of
    its kind at its full height, and strided ones also at a partial height."""
    import paper_1607_01039_amd as F
    cases = []
    for v in F.list_variants(dtype):
        base = v[:-1] if v.endswith("n") else v  # "n": twin with non-temporal loads and stores
        held = base.endswith("p")  # "p": held in registers, two workgroups per CU
        wide = base.endswith("w")  # "w": the same tile in twice the threads
        core = base[:-1] if held or wide else base
        if core.startswith("C"):
            tb = int(core[1:])
            if core == "C16" or held:  # only as a first pass over all its bits
                s4, s1 = ("S11c7:4", "S8c7:1") if dtype == "int64" else ("S12c8:4", "S9c8:1")
                cases.append((v, tb + 4, f"{v},{s4}"))
                cases.append((v, tb + 1, f"{v},{s1}"))
            else:
                cases.append((v, tb, v))
                cases.append((v, tb - 3, v))
        else:
            tb, cb = (int(x) for x in core[1:].split("c"))
            R = tb - cb
            cases.append((v, 12 + R, f"C12,{v}:{R}"))
            whole = held or (1 << tb) * (8 if dtype == "int64" else 4) == 256 * 1024
            if R > 1 and not whole:  # register-resident strided tiles: full height only
                cases.append((v, 12 + R - 1, f"C12,{v}:{R - 1}"))
    return cases


def _cases_or_empty(dtype):
    try:
        return _variant_cases(dtype)
    except Exception:  # library not built: the test itself will fail loudly
        return [("unbuilt", 0, "")]


@pytest.mark.parametrize("variant,n,spec", _cases_or_empty("int32"))
def test_every_variant_int32(F, O, variant, n, spec):
    x = synth.ints(1 << n, 40 + n, -(1 << 20), 1 << 20, dtype=np.int32)
    F.set_schedule("int32", n, spec)
    try:
        y, _ = _run_int(F, x)
    finally:
        F.set_schedule("int32", n, None)
    assert np.array_equal(y, O.wht_fig1(x))


@pytest.mark.parametrize("variant,n,spec", _cases_or_empty("int64"))
def test_every_variant_int64(F, O, variant, n, spec):
    x = synth.ints(1 << n, 50 + n, -(1 << 40), 1 << 40, dtype=np.int64)
    F.set_schedule("int64", n, spec)
    try:
        y, _ = _run_int(F, x)
    finally:
        F.set_schedule("int64", n, None)
    assert np.array_equal(y, O.wht_fig1(x))


@pytest.mark.parametrize("n,spec", [(n, s) for n, ss in SCHEDULES_I32.items() for s in ss])
def test_every_schedule_gives_the_same_bits_i32(F, O, n, spec):
    x = synth.signs(1 << n, 5 + n)
    F.set_schedule("int32", n, spec)
    try:
        y, _ = _run_int(F, x)
    finally:
        F.set_schedule("int32", n, None)
    assert np.array_equal(y, O.wht_fig2(x, 3))


@pytest.mark.parametrize("n,spec", [(n, s) for n, ss in SCHEDULES_I64.items() for s in ss])
def test_every_schedule_gives_the_same_bits_i64(F, O, n, spec):
    x = synth.ints(1 << n, 6 + n, -(1 << 35), 1 << 35, dtype=np.int64)
    F.set_schedule("int64", n, spec)
    try:
        y, _ = _run_int(F, x)
    finally:
        F.set_schedule("int64", n, None)
    assert np.array_equal(y, O.wht_fig1(x))


def test_config_n24_signs(F, O):
    # +-1 signs, n = 24, seed 1: full element-by-element parity.
    x = synth.signs(1 << 24, 1)
    y, _ = _run_int(F, x)
    assert np.array_equal(y, O.wht_fig2(x, 3))


@pytest.mark.parametrize("n,p,seed,T", [(16, 0.45, 2, 6 * 256), (18, 0.3, 3, 4 * 512), (21, 0.45, 4, 5 * 1448),
                                        (13, 0.45, 5, -1), (12, 0.45, 6, 0)])
def test_fused_threshold_matches_oracle(F, O, n, p, seed, T):
    x, s, err = synth.planted(n, seed, p)
    y, hits = _run_int(F, x, threshold=T, cap=1 << n)
    ref = O.wht_fig1(x)
    assert np.array_equal(y, ref)
    ridx, rval, rcnt = O.threshold(ref, T)
    assert hits.count == rcnt
    gi, gv = hits.sorted()
    assert np.array_equal(gi, ridx.astype(np.int64)) and np.array_equal(gv, rval)
    if T >= 0 and T < (1 << n) - 2 * err:
        assert s in set(gi.tolist())


def _register_strided_int32():
    import paper_1607_01039_amd as F
    try:
        names = F.list_variants("int32")
    except Exception:  # library not built: the test itself will fail loudly
        return ["unbuilt"]
    return [v for v in names if v.startswith("S16") or (v.startswith("S") and v.rstrip("n").endswith("p"))]


@pytest.mark.parametrize("variant", _register_strided_int32())
def test_fused_threshold_register_strided(F, O, variant):
    """The threshold fused into a register-resident strided pass (2^16-entry
    tiles in 1024 threads, 2^15-entry tiles in 512) as the last pass: every
    entry, the hit set and the hit values against the oracle."""
    core = variant[:-1] if variant.endswith("n") else variant
    tb, cb = (int(x) for x in core[1:].rstrip("p").split("c"))
    R = tb - cb
    n = 12 + R
    x, s, err = synth.planted(n, 70 + n, 0.4)
    T = 4 << (n // 2)
    F.set_schedule("int32", n, f"C12,{variant}:{R}")
    try:
        y, hits = _run_int(F, x, threshold=T, cap=1 << n)
    finally:
        F.set_schedule("int32", n, None)
    ref = O.wht_fig1(x)
    assert np.array_equal(y, ref)
    ridx, rval, rcnt = O.threshold(ref, T)
    assert rcnt > 1 and hits.count == rcnt
    gi, gv = hits.sorted()
    assert np.array_equal(gi, ridx.astype(np.int64)) and np.array_equal(gv, rval)
    assert s in set(gi.tolist())


def _wide_int64():
    import paper_1607_01039_amd as F
    try:
        names = F.list_variants("int64")
    except Exception:  # library not built: the test itself will fail loudly
        return ["unbuilt"]
    return [v for v in names if v.rstrip("n").endswith("w")]


@pytest.mark.parametrize("variant", _wide_int64())
def test_fused_threshold_wide_int64(F, O, variant):
    """The threshold fused into an 8-byte strided tile held by 1024 threads
    as the last pass: every entry, the hit set and the hit values against the
    oracle."""
    core = variant.rstrip("n")[:-1]
    tb, cb = (int(x) for x in core[1:].split("c"))
    R = tb - cb
    n = 12 + R
    x, s, err = synth.planted(n, 90 + n, 0.4, dtype=np.int64)
    T = 4 << (n // 2)
    F.set_schedule("int64", n, f"C12,{variant}:{R}")
    try:
        y, hits = _run_int(F, x, threshold=T, cap=1 << n)
    finally:
        F.set_schedule("int64", n, None)
    ref = O.wht_fig1(x)
    assert np.array_equal(y, ref)
    ridx, rval, rcnt = O.threshold(ref, T)
    assert rcnt > 1 and hits.count == rcnt
    gi, gv = hits.sorted()
    assert np.array_equal(gi, ridx.astype(np.int64)) and np.array_equal(gv, rval)
    assert s in set(gi.tolist())


@pytest.mark.parametrize("n", [12, 20, 30])
def test_reused_hit_buffers(F, O, n):
    """The library clears the hit count itself (inside the first of several
    passes, or with a launch of its own for a single pass): the same output
    buffers reused across calls, still holding the previous call's hits, give
    each call exactly its own hits."""
    import torch
    x, s, err = synth.planted(n, 11 + n, 0.3)
    T = (6 if n >= 30 else 4) << (n // 2)  # about 14 noise hits at n = 20, none expected at n = 30
    src = _dev(x)
    t = torch.empty_like(src)
    bufs = F.hit_buffers(t, 1 << 12)
    if n <= 20:
        ridx, rval, rcnt = O.threshold(O.wht_fig1(x), T)
    for rep in range(3):
        t.copy_(src)
        out = F.fwht_int_(t, threshold=T, sync=False, hits=bufs)
        assert out is bufs
        torch.cuda.synchronize()
        hits = F._collect(*bufs, 1 << 12)
        gi, gv = hits.sorted()
        if n <= 20:
            assert hits.count == rcnt and np.array_equal(gi, ridx.astype(np.int64)) and np.array_equal(gv, rval)
        else:  # n = 30: the planted peak and its exact value; each hit checked by a direct sum
            assert s in set(gi.tolist()) and int(gv[list(gi).index(s)]) == (1 << n) - 2 * err
            if rep == 0:
                ks = gi[:2].tolist()
                assert np.array_equal(O.wht_def_at(x, ks), gv[:2].astype(np.int64))


def test_fused_threshold_capacity_overflow(F, O):
    n = 12
    x = synth.signs(1 << n, 9)
    y, hits = _run_int(F, x, threshold=-1, cap=100)
    assert hits.count == 1 << n and len(hits.idx) == 100
    ref = O.wht_fig1(x)
    assert np.array_equal(ref[hits.idx], hits.val)
    assert len(set(hits.idx.tolist())) == 100


def test_int64_threshold(F, O):
    n = 17
    x, s, err = synth.planted(n, 8, 0.4, dtype=np.int64)
    y, hits = _run_int(F, x, threshold=(1 << n) // 8, cap=4096)
    ref = O.wht_fig1(x)
    assert np.array_equal(y, ref)
    ridx, rval, rcnt = O.threshold(ref, (1 << n) // 8)
    gi, gv = hits.sorted()
    assert hits.count == rcnt and np.array_equal(gi, ridx.astype(np.int64)) and np.array_equal(gv, rval)


@pytest.mark.parametrize("n", [0, 2, 5, 11, 12, 19])
@pytest.mark.parametrize("dtype", [np.int32, np.int64, np.float32])
def test_standalone_threshold(F, O, dtype, n):
    """Blocks of 4 x 256 16-byte vectors: n = 19 is whole blocks, n <= 11 only
    the bounds-checked partial block (one block for int32 at n = 12)."""
    if dtype == np.float32:
        x = synth.normal(1 << n, 3) * 4
        T = 9.5
    else:
        x = synth.ints(1 << n, 3, -1000, 1000, dtype=dtype)
        T = 990
    if n >= 3:
        x[5] = T
        x[6] = -T
    x[0] = -2 * T  # a hit in the first entry at every size
    hits = F.threshold(_dev(x), T, cap=1 << 14)
    ridx, rval, rcnt = O.threshold(x, T)
    gi, gv = hits.sorted()
    assert hits.count == rcnt and np.array_equal(gi, ridx.astype(np.int64)) and np.array_equal(gv, rval.astype(dtype))
    assert 5 not in set(gi.tolist()) and 0 in set(gi.tolist())


def test_repeat_runs_bit_identical(F):
    n = 22
    x = synth.signs(1 << n, 11)
    outs = [_run_int(F, x)[0] for _ in range(3)]
    assert all(np.array_equal(outs[0], o) for o in outs[1:])


def test_involution_on_gpu(F):
    n = 23
    x = synth.ints(1 << n, 12, -100, 100, dtype=np.int32)
    t = _dev(x)
    F.fwht_int_(t)
    F.fwht_int_(t)
    assert np.array_equal(t.cpu().numpy(), x * (1 << n))


def test_config_n30_planted_sampled(F, O):
    """n = 30 planted peak (seed 2, p = 0.45, T = 6 * 2^15) in the bench's launch
    configuration: closed-form peak, definition at sampled k, threshold set,
    and full element-by-element parity against the multi-threaded Fig. 2."""
    import torch
    n, T = 30, 6 * (1 << 15)
    x, s, err = synth.planted(n, 2, 0.45)
    t = _dev(x)
    hits = F.fwht_int_(t, threshold=T, cap=1 << 16)
    y = t.cpu().numpy()
    del t
    torch.cuda.empty_cache()
    assert int(y[s]) == (1 << n) - 2 * err
    rng = np.random.default_rng(0)
    ks = [0, s, (1 << n) - 1] + [int(k) for k in rng.integers(0, 1 << n, size=3)]
    assert np.array_equal(O.wht_def_at(x, ks), y[ks].astype(np.int64))
    ridx, rval, rcnt = O.threshold(y, T)
    gi, gv = hits.sorted()
    assert hits.count == rcnt and np.array_equal(gi, ridx.astype(np.int64)) and np.array_equal(gv, rval)
    assert s in set(gi.tolist())
    O.wht_fig2_inplace(x, 4)
    assert np.array_equal(y, x)


@pytest.mark.parametrize("nbytes", [16, 4096 + 16, 64 << 20])
def test_copy_kernel(F, nbytes):
    """The library's copy kernel (the bandwidth and counter calibration
    reference) copies exactly, for a single vector, a ragged grid tail and
    many blocks."""
    import torch
    src = _dev(synth.ints(nbytes // 4, 77, -(1 << 30), 1 << 30, dtype=np.int32))
    dst = torch.zeros_like(src)
    F.copy_(dst, src)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)


# ---- the tuned default schedules, element by element --------------------------
#
# Every size from 2^13 entries up runs the schedule of the tuned table
# (tune/gfx950.txt) unless a test overrides it; these tests run that default
# at every such size and compare every entry with the oracle's Fig. 2 (16
# host threads), so that a retuned table cannot change a result unnoticed.

def _tuned_table():
    import os
    import paper_1607_01039_amd as F
    path = os.path.join(os.path.dirname(F.__file__), "tune", "gfx950.txt")
    tab = {}
    for ln in open(path):
        f = ln.split()
        if f and not ln.startswith("#") and f[0] != "batched":
            tab[(f[0], int(f[1]))] = f[2]
    return tab


CHUNK = 1 << 27  # entries per host <-> device copy and per comparison


def _upload(x):
    import torch
    t = torch.empty(x.size, dtype=torch.from_numpy(x[:1]).dtype, device="cuda")
    for c0 in range(0, x.size, CHUNK):
        t[c0:c0 + CHUNK].copy_(torch.from_numpy(x[c0:c0 + CHUNK]))
    return t


def _equal_chunks(t, ref):
    """Device tensor t equals the host array ref entry for entry (chunked, so
    no second full-size host copy is made); returns the first bad chunk."""
    for c0 in range(0, ref.size, CHUNK):
        if not np.array_equal(t[c0:c0 + CHUNK].cpu().numpy(), ref[c0:c0 + CHUNK]):
            return c0
    return None


def _default_schedule_parity(F, O, dtype_name, n, x):
    import torch
    tab = _tuned_table()
    if (dtype_name, n) in tab:
        assert F.get_schedule(dtype_name, n) == tab[(dtype_name, n)]
    print(f"{dtype_name} n={n} schedule {F.get_schedule(dtype_name, n)}", flush=True)
    t = _upload(x)
    F.fwht_int_(t)
    torch.cuda.synchronize()
    O.wht_fig2_inplace(x, 4)  # x becomes the expected transform
    bad = _equal_chunks(t, x)
    del t
    torch.cuda.empty_cache()
    assert bad is None, f"first differing chunk at entry {bad}"


@pytest.mark.parametrize("n", list(range(23, 30)))
def test_int32_default_schedule(F, O, n):
    # full-range int32 values: every entry wraps mod 2^32
    x = synth.ints(1 << n, 4000 + n, -(1 << 31), (1 << 31) - 1, dtype=np.int32)
    _default_schedule_parity(F, O, "int32", n, x)


@pytest.mark.parametrize("n", list(range(13, 33)))
def test_int64_default_schedule(F, O, n):
    # full-range int64 values (every bit random): every entry wraps mod 2^64;
    # n = 32 is 32 GiB on each side
    x = synth.raw64(1 << n, 4100 + n)
    _default_schedule_parity(F, O, "int64", n, x)


@pytest.mark.parametrize("n,spec", [(29, "C14pn,S14c5n:9,S13c6:5,S12c6:1"), (30, "C14pn,S14c5n:9,S13c6:5,S12c6:2")])
def test_int64_lane_offset_boundary(F, O, n, spec):
    """A strided tile pass keeps lane offsets in 32 bits: S12c6 (one row bit
    among its lane bits) at row stride 2^28 is the largest accepted stride for
    8-byte entries (2^28 * 8 = 2^31 bytes), and every entry must still match
    the oracle there; one bit further up the library refuses it."""
    import torch
    x = synth.raw64(1 << n, 4300 + n)
    F.set_schedule("int64", n, spec)
    try:
        t = _upload(x)
        F.fwht_int_(t)
        torch.cuda.synchronize()
    finally:
        F.set_schedule("int64", n, None)
    O.wht_fig2_inplace(x, 4)
    bad = _equal_chunks(t, x)
    del t
    torch.cuda.empty_cache()
    assert bad is None, f"first differing chunk at entry {bad}"
    with pytest.raises(F.FWHTError, match="lane offsets"):
        F.set_schedule("int64", 30, "C14pn,S14c5n:9,S13c6:6,S12c6:1")  # S12c6 at 2^29


# n = 35 holds 256 GiB in HBM and 256 GiB of host memory for the oracle's copy,
# close to what one process may use on the host, so it runs only on request
_N35 = pytest.param(35, marks=pytest.mark.skipif(
    os.environ.get("FWHT_TEST_N35") != "1",
    reason="256 GiB on the device and on the host; set FWHT_TEST_N35=1 to run"))


@pytest.mark.parametrize("n", [33, 34, _N35])
def test_int64_large_in_hbm(F, O, n):
    """int64 up to the in-HBM limit (n = 35: 256 GiB resident), planted peak
    (seed 3, p = 0.48), fused threshold T = ceil(6 * 2^(n/2)): every entry
    against the oracle's Fig. 2 run in place on the host copy of the input,
    the hit set against the oracle's threshold scan, the peak in closed form,
    and the randomized Kronecker-weight identity (independent of Fig. 2)."""
    import math
    import torch
    N = 1 << n
    T = int(math.ceil(6 * 2 ** (n / 2)))
    print(f"int64 in HBM n={n}: generating", flush=True)
    x, s, err = synth.planted(n, 3, 0.48, dtype=np.int64)
    # the randomized identity sum_k W_k w_k = sum_i x_i (H w)_i (mod 2^61 - 1)
    # for Kronecker-product weights, input side taken before Fig. 2 runs in place
    tw = [int(v) for v in np.random.default_rng(n).integers(0, O.KF_P, size=n, dtype=np.uint64)]
    kf_in = O.kf_sum(x, n, tw, 1)
    t = _upload(x)
    print("transforming", flush=True)
    hits = F.fwht_int_(t, threshold=T, cap=1 << 12)
    assert int(t[s].item()) == N - 2 * err
    kf_out = sum(O.kf_sum(t[c0:c0 + CHUNK].cpu().numpy(), n, tw, 0, start=c0) for c0 in range(0, N, CHUNK)) % O.KF_P
    assert kf_out == kf_in
    print("oracle (Fig. 2, 16 threads)", flush=True)
    O.wht_fig2_inplace(x, 4)
    print("comparing", flush=True)
    bad = _equal_chunks(t, x)
    del t
    torch.cuda.empty_cache()
    assert bad is None, f"first differing chunk at entry {bad}"
    ridx, rval, rcnt = O.threshold(x, T, cap=1 << 12)
    gi, gv = hits.sorted()
    assert hits.count == rcnt and np.array_equal(gi, ridx.astype(np.int64)) and np.array_equal(gv, rval)
    assert s in set(gi.tolist())
