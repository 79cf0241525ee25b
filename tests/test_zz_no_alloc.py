"""hg_hegmm_noalloc: the product computed in the library's fixed per-GPU
workspace, with no device allocation, equals hg_hegmm's bit for bit."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2405_02238_amd as hg  # noqa: E402


def _operands(ctx, shape, seed, nonce):
    m, l, n = shape
    rng = np.random.default_rng(seed)
    A = rng.integers(-8, 9, size=(m, l))
    B = rng.integers(-8, 9, size=(l, n))
    return A, B, ctx.encrypt(0, A, m, l, n, nonce=nonce), ctx.encrypt(1, B, m, l, n, nonce=nonce)


def test_noalloc_equals_hegmm_twice_then_smaller():
    """Two calls in a row into one result handle: the full 64x32x48 product
    at N = 8192, then a smaller 16x8x24 one; each equals hg_hegmm's result
    for the same operands bit for bit and decrypts to A.B mod t."""
    c = workloads.HEADLINE
    big, small = (64, 32, 48), (16, 8, 24)
    ctx = hg.Context(c.N, c.t, c.L, c.alpha)
    ctx.keygen(c.seed, [big, small])
    A, B = workloads.headline_operands()
    ca, cb = ctx.encrypt(0, A, *big, nonce=1), ctx.encrypt(1, B, *big, nonce=1)
    want_big = ctx.hegmm(ca, cb, *big).export()
    out = ctx.import_ct(np.zeros(2 * c.L * c.N, dtype=np.uint64), 1, 2)
    ctx.hegmm_noalloc(ca, cb, *big, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.export(), want_big)
    assert np.array_equal(ctx.decrypt(out, *big), workloads.plain_matmul_mod(A, B, c.t))
    A2, B2, ca2, cb2 = _operands(ctx, small, 7, 2)
    want_small = ctx.hegmm(ca2, cb2, *small).export()
    ctx.hegmm_noalloc(ca2, cb2, *small, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.export(), want_small)
    assert np.array_equal(ctx.decrypt(out, *small), workloads.plain_matmul_mod(A2, B2, c.t))
    # the workspace keeps the last call's contents; a repeat of the big
    # product over them is still exact
    ctx.hegmm_noalloc(ca, cb, *big, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.export(), want_big)


def test_noalloc_fold_transposed_and_errors():
    """Plans with a fold and with transposition at N = 1024 equal hg_hegmm's
    bits; a product whose workspace exceeds the fixed array, an unprepared
    shape, and an operand as result handle are refused without running."""
    c = workloads.TINY
    shapes = [(2, 5, 7), (5, 4, 2), (3, 11, 6)]
    ctx = hg.Context(c.N, c.t, c.L, c.alpha)
    ctx.keygen(c.seed, shapes)
    out = ctx.import_ct(np.zeros(2 * c.L * c.N, dtype=np.uint64), 1, 2)
    for i, s in enumerate(shapes):
        A, B, ca, cb = _operands(ctx, s, 30 + i, 5 + i)
        want = ctx.hegmm(ca, cb, *s).export()
        ctx.hegmm_noalloc(ca, cb, *s, out)
        torch.cuda.synchronize()
        assert np.array_equal(out.export(), want), s
        assert np.array_equal(ctx.decrypt(out, *s), workloads.plain_matmul_mod(A, B, c.t)), s
    with pytest.raises(hg.HGError) as e:
        ctx.hegmm_noalloc(ca, cb, 9, 9, 9, out)
    assert e.value.code == hg.HG_ESTATE
    with pytest.raises(hg.HGError) as e:
        ctx.hegmm_noalloc(ca, cb, *shapes[-1], ca)
    assert e.value.code == hg.HG_EINVAL
    # the paper-order composition of the headline product divides each of
    # its 124 rotations by P on its own: about 170 MB of workspace
    h = workloads.HEADLINE
    big = (64, 32, 48)
    wide = hg.Context(h.N, h.t, h.L, h.alpha, ks_order=1)
    wide.keygen(h.seed, [big])
    A, B = workloads.headline_operands()
    ca, cb = wide.encrypt(0, A, *big, nonce=1), wide.encrypt(1, B, *big, nonce=1)
    res = wide.import_ct(np.zeros(2 * h.L * h.N, dtype=np.uint64), 1, 2)
    before = res.export()
    with pytest.raises(hg.HGError) as e:
        wide.hegmm_noalloc(ca, cb, *big, res)
    assert e.value.code == hg.HG_EINVAL and "workspace" in str(e.value)
    torch.cuda.synchronize()
    assert np.array_equal(res.export(), before)
    # the context still works for the allocating entry point afterwards
    assert np.array_equal(wide.decrypt(wide.hegmm(ca, cb, *big), *big), workloads.plain_matmul_mod(A, B, h.t))
