"""GPU parity of the FP32 float transform against the FP64 oracle.

Tolerance (derived from the arithmetic): each of the n radix-2 stages rounds
every entry once to FP32 (unit roundoff u = 2^-24), and the stages are
orthogonal up to a factor sqrt(2), so the normwise relative error of the
unnormalised result is at most about n * u * sqrt(2) plus one rounding of the
scale.  The tests gate at (n + 2) * 2^-23, twice that bound.
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


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def tol(n):
    return (n + 2) * 2.0 ** -23


def normwise(y, ref):
    y = y.reshape(-1, ref.shape[-1]).astype(np.float64)
    r = ref.reshape(-1, ref.shape[-1])
    return float(np.max(np.linalg.norm(y - r, axis=1) / np.maximum(np.linalg.norm(r, axis=1), 1e-300)))


@pytest.mark.parametrize("n,batch", [(0, 5), (1, 3), (2, 1), (3, 7), (5, 33), (8, 3), (11, 2), (12, 5),
                                     (13, 3), (14, 2), (15, 1), (16, 3), (19, 1), (20, 2), (22, 1)])
@pytest.mark.parametrize("normalize", [True, False])
def test_float_matches_oracle(F, O, n, batch, normalize):
    x = synth.normal((batch, 1 << n), 100 * n + batch)
    t = _dev(x)
    F.fwht_float_(t, normalize=normalize)
    ref = O.wht_batch(x, n, normalize)
    assert normwise(t.cpu().numpy(), ref) <= tol(n)


@pytest.mark.parametrize("n", list(range(13, 29)))
def test_float_default_schedule(F, O, n):
    """The tuned default schedule of every size of the table (n = 13..28), one
    transform per row, two rows up to n = 26, against the FP64 oracle."""
    batch = 2 if n <= 26 else 1
    x = synth.normal((batch, 1 << n), 500 + n)
    print(f"float32 n={n} schedule {F.get_schedule('float32', n)}", flush=True)
    t = _dev(x)
    F.fwht_float_(t, normalize=True)
    y = t.cpu().numpy()
    del t
    assert normwise(y, O.wht_batch(x, n, True)) <= tol(n)


def test_float_config_autograd_shape(F, O):
    # 256 x 2^20 orthonormal (the autograd workload), sampled rows vs the oracle.
    n, B = 20, 256
    x = synth.normal((B, 1 << n), 5)
    t = _dev(x)
    F.fwht_float_(t, normalize=True)
    y = t.cpu().numpy()
    for r in (0, 77, 255):
        ref = O.wht_batch(x[r:r + 1], n, True)
        assert normwise(y[r:r + 1], ref) <= tol(n)
    # Parseval per row
    assert np.allclose((y.astype(np.float64) ** 2).sum(1), (x.astype(np.float64) ** 2).sum(1), rtol=1e-5)


def test_float_integer_inputs_exact(F, O):
    # Small-integer inputs stay exactly representable: bit-exact, unnormalised.
    n = 18
    x = synth.ints(1 << n, 4, -8, 8, dtype=np.int64).astype(np.float32)
    t = _dev(x)
    F.fwht_float_(t, normalize=False)
    assert np.array_equal(t.cpu().numpy().astype(np.float64), O.wht_fig1(x))


def _float_variant_cases():
    import paper_1607_01039_amd as F
    try:
        vs = F.list_variants("float32")
    except Exception:
        return [("unbuilt", 0, "")]
    cases = []
    for v in vs:
        base = v[:-1] if v.endswith("n") else v  # "n": twin with non-temporal loads and stores
        held = base.endswith("p")  # "p": held in registers, two workgroups per CU
        core = base[:-1] if held else base
        if core.startswith("C"):
            if core == "C16" or held:  # only as a first pass over all its bits
                cases.append((v, int(core[1:]) + 4, f"{v},S12c8:4"))
            else:
                cases.append((v, int(core[1:]), v))
        else:
            tb, cb = (int(x) for x in core[1:].split("c"))
            cases.append((v, 12 + tb - cb, f"C12,{v}:{tb - cb}"))
    return cases


@pytest.mark.parametrize("variant,n,spec", _float_variant_cases())
def test_every_variant_float(F, O, variant, n, spec):
    x = synth.normal((2, 1 << n), 60 + n)
    F.set_schedule("float32", n, spec)
    try:
        t = _dev(x)
        F.fwht_float_(t, normalize=True)
        y = t.cpu().numpy()
    finally:
        F.set_schedule("float32", n, None)
    assert normwise(y, O.wht_batch(x, n, True)) <= tol(n)


@pytest.mark.parametrize("n,batch", [(0, 3), (1, 2), (2, 5), (5, 7), (12, 3), (13, 2), (16, 2), (17, 1), (20, 3),
                                     (22, 1), (24, 1)])
@pytest.mark.parametrize("normalize", [True, False])
def test_float_out_of_place(F, O, n, batch, normalize):
    """fwht_float_out: the first pass reads src and writes dst; the result must
    equal the in-place transform bit for bit, src must be untouched, and the
    result must meet the oracle bound."""
    import torch
    x = synth.normal((batch, 1 << n), 700 + 10 * n + batch)
    src = _dev(x)
    out = F.fwht_float_out(src, normalize=normalize)
    ref_t = _dev(x)
    F.fwht_float_(ref_t, normalize=normalize)
    torch.cuda.synchronize()
    assert np.array_equal(src.cpu().numpy(), x)
    y = out.cpu().numpy()
    assert np.array_equal(y, ref_t.cpu().numpy())
    assert normwise(y, O.wht_batch(x, n, normalize)) <= tol(n)


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_float_out_of_place_matrix_cores(F, prec):
    """The matrix-core precisions copy src to dst and transform in place: the
    same bits as fwht_float_ on a copy."""
    import torch
    x = synth.normal((4, 1 << 12), 801)
    src = _dev(x)
    out = torch.empty_like(src)
    F.fwht_float_out(src, out, True, prec)
    ref_t = _dev(x)
    F.fwht_float_(ref_t, True, prec)
    torch.cuda.synchronize()
    assert np.array_equal(src.cpu().numpy(), x)
    assert np.array_equal(out.cpu().numpy(), ref_t.cpu().numpy())
