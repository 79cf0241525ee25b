"""GPU: error paths of the C ABI and the client/server roles."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2405_02238_amd as hg  # noqa: E402


@pytest.fixture()
def ctx():
    c = workloads.TINY
    x = hg.Context(c.N, c.t, c.L, c.alpha)
    x.keygen(c.seed, [(4, 3, 5)])
    return x


def test_bad_parameters():
    with pytest.raises(hg.HGError) as e:
        hg.Context(1000, 12289, 3, 1)          # N not a power of two
    assert e.value.code == hg.HG_EINVAL
    with pytest.raises(hg.HGError) as e:
        hg.Context(1024, 12288, 3, 1)          # t not prime
    assert e.value.code == hg.HG_EINVAL
    with pytest.raises(hg.HGError) as e:
        hg.Context(1024, 65539, 3, 1)          # t prime but not 1 mod 2N
    assert e.value.code == hg.HG_EINVAL


def test_dimensions_and_fit(ctx):
    A, B = workloads.tiny_operands()
    with pytest.raises(hg.HGError) as e:
        ctx.encrypt(0, A, 0, 3, 5)
    assert e.value.code == hg.HG_EINVAL
    # m * n alone exceeds the 512 slots: no inner blocking can fit it
    with pytest.raises(hg.HGError) as e:
        ctx.plan_info(30, 4, 30)
    assert e.value.code == hg.HG_ENOFIT


def test_missing_rotation_keys(ctx):
    rng = np.random.default_rng(0)
    m, l, n = 3, 7, 5                            # not listed in keygen
    A = rng.integers(-8, 9, size=(m, l))
    B = rng.integers(-8, 9, size=(l, n))
    ca, cb = ctx.encrypt(0, A, m, l, n, nonce=1), ctx.encrypt(1, B, m, l, n, nonce=1)
    with pytest.raises(hg.HGError) as e:
        ctx.hegmm(ca, cb, m, l, n)
    assert e.value.code == hg.HG_ENOKEY
    ctx.keygen(workloads.TINY.seed, [(m, l, n)])  # adding keys later under the same seed
    C = ctx.decrypt(ctx.hegmm(ca, cb, m, l, n), m, l, n)
    assert np.array_equal(C, workloads.plain_matmul_mod(A, B, workloads.TINY.t))
    with pytest.raises(hg.HGError) as e:
        ctx.keygen(workloads.TINY.seed + 1, [(m, l, n)])   # another seed
    assert e.value.code == hg.HG_ESTATE


def test_mismatched_operands(ctx):
    A, B = workloads.tiny_operands()
    ca, cb = ctx.encrypt(0, A, 4, 3, 5, nonce=2), ctx.encrypt(1, B, 4, 3, 5, nonce=2)
    with pytest.raises(hg.HGError) as e:
        ctx.hegmm(cb, ca, 4, 3, 5)               # roles swapped
    assert e.value.code == hg.HG_EINVAL
    with pytest.raises(hg.HGError) as e:
        ctx.hegmm(ca, cb, 4, 3, 6)               # other shape
    assert e.value.code in (hg.HG_EINVAL, hg.HG_ENOKEY)
    cc = ctx.hegmm(ca, cb, 4, 3, 5)
    with pytest.raises(hg.HGError) as e:
        ctx.decrypt(cc, 5, 3, 4)                 # result of another shape
    assert e.value.code == hg.HG_EINVAL
    with pytest.raises(hg.HGError) as e:
        ctx.decrypt(ca, 4, 3, 5)                 # a packed operand, not a result
    assert e.value.code == hg.HG_EINVAL


def test_server_role_after_drop_secret(ctx):
    """The cloud keeps only evaluation keys: products still run, encryption
    and decryption are refused, and the client (who keeps the secret in its
    own context) decrypts the exported result."""
    A, B = workloads.tiny_operands()
    c = workloads.TINY
    client = hg.Context(c.N, c.t, c.L, c.alpha)
    client.keygen(c.seed, [(4, 3, 5)])
    wa = client.encrypt(0, A, 4, 3, 5, nonce=3).export()
    wb = client.encrypt(1, B, 4, 3, 5, nonce=3).export()
    ctx.drop_secret()
    with pytest.raises(hg.HGError) as e:
        ctx.encrypt(0, A, 4, 3, 5, nonce=4)
    assert e.value.code == hg.HG_ESTATE
    ca, cb = ctx.import_ct(wa, 1, 2), ctx.import_ct(wb, 1, 2)
    # imported operands carry no shape: the product refuses them until they
    # come from hg_encrypt for that shape
    with pytest.raises(hg.HGError):
        ctx.hegmm(ca, cb, 4, 3, 5)
    with pytest.raises(hg.HGError) as e:
        ctx.decrypt_slots(ca)
    assert e.value.code == hg.HG_ESTATE
    # the evaluation path through the server accepts serialised operands
    with hg.Server(ctx, max_batch=2, lanes=1) as srv:
        words, _ = srv.wait(srv.submit(wa, wb, 4, 3, 5))
    C = client.decrypt(client.import_ct(words, 1, 2), 4, 3, 5)
    assert np.array_equal(C, workloads.plain_matmul_mod(A, B, c.t))


def test_export_buffer_and_import_checks(ctx):
    A, B = workloads.tiny_operands()
    ca = ctx.encrypt(0, A, 4, 3, 5, nonce=5)
    w = ca.export()
    bad = w.copy()
    bad[0] = np.uint64(2 ** 62)                  # residue out of range
    with pytest.raises(hg.HGError) as e:
        ctx.import_ct(bad, 1, 2)
    assert e.value.code == hg.HG_EINVAL
    with pytest.raises(hg.HGError) as e:
        ctx.import_ct(w[:-1], 1, 2)              # wrong length
    assert e.value.code == hg.HG_EINVAL


def test_repeat_and_stream_determinism(ctx):
    """The same product twice, on the null stream and on a second stream,
    gives the same bits."""
    A, B = workloads.tiny_operands()
    ca, cb = ctx.encrypt(0, A, 4, 3, 5, nonce=6), ctx.encrypt(1, B, 4, 3, 5, nonce=6)
    first = ctx.hegmm(ca, cb, 4, 3, 5).export()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        other = ctx.hegmm(ca, cb, 4, 3, 5)
    s.synchronize()
    assert np.array_equal(other.export(), first)
    assert np.array_equal(ctx.hegmm(ca, cb, 4, 3, 5).export(), first)


def test_back_to_back_products_through_the_staging_ring():
    """24 products of alternating shapes and operands enqueued back to back
    on one stream with no synchronisation: the host stages each call's
    descriptor tables in the next slot of its ring while the device may
    still be copying out of earlier ones (only every eighth copy is waited
    for), three times round the ring.  Each result equals the same product
    computed on its own."""
    c = workloads.TINY
    shapes = [(4, 3, 5), (2, 5, 7), (5, 4, 2)]
    ctx = hg.Context(c.N, c.t, c.L, c.alpha)
    ctx.keygen(c.seed, shapes)
    rng = np.random.default_rng(24)
    ops = []
    for i, (m, l, n) in enumerate(shapes * 2):
        A, B = rng.integers(-8, 9, size=(m, l)), rng.integers(-8, 9, size=(l, n))
        ops.append(((m, l, n), ctx.encrypt(0, A, m, l, n, nonce=90 + i), ctx.encrypt(1, B, m, l, n, nonce=90 + i)))
    alone = []
    for shape, a, b in ops:
        alone.append(ctx.hegmm(a, b, *shape).export())
        torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        outs = [ctx.hegmm(ops[i % len(ops)][1], ops[i % len(ops)][2], *ops[i % len(ops)][0]) for i in range(24)]
    s.synchronize()
    for i, o in enumerate(outs):
        assert np.array_equal(o.export(), alone[i % len(ops)]), i


def test_batch_rejects_before_any_work(ctx):
    """A batch with one request that cannot run (no rotation keys for its
    shape) is refused as a whole before anything is enqueued; the same
    batch without it then gives the bits of each product alone."""
    A, B = workloads.tiny_operands()
    rng = np.random.default_rng(1)
    A2, B2 = rng.integers(-8, 9, size=(3, 7)), rng.integers(-8, 9, size=(7, 5))
    ca, cb = ctx.encrypt(0, A, 4, 3, 5, nonce=7), ctx.encrypt(1, B, 4, 3, 5, nonce=7)
    ca2, cb2 = ctx.encrypt(0, A2, 3, 7, 5, nonce=7), ctx.encrypt(1, B2, 3, 7, 5, nonce=7)
    alone = ctx.hegmm(ca, cb, 4, 3, 5).export()
    torch.cuda.synchronize()
    with pytest.raises(hg.HGError) as e:
        ctx.hegmm_batch([ca, ca2], [cb, cb2], [(4, 3, 5), (3, 7, 5)])
    assert e.value.code == hg.HG_ENOKEY
    with pytest.raises(hg.HGError) as e:
        ctx.hegmm_batch([ca, cb], [cb, ca], [(4, 3, 5), (4, 3, 5)])   # roles swapped in the second
    assert e.value.code == hg.HG_EINVAL
    out = ctx.hegmm_batch([ca, ca], [cb, cb], [(4, 3, 5), (4, 3, 5)])
    for c in out:
        assert np.array_equal(c.export(), alone)


def test_caller_allocator():
    """Handles from the caller's allocator (torch's caching allocator) hold
    the same bits as library-allocated ones, on any stream; their memory is
    torch's and returns to it when they are freed, also after the allocator
    was switched back to hipMalloc."""
    import gc
    c = workloads.TINY
    A, B = workloads.tiny_operands()
    ctx = hg.Context(c.N, c.t, c.L, c.alpha)
    ctx.keygen(c.seed, [(4, 3, 5)])
    ref = ctx.hegmm(ctx.encrypt(0, A, 4, 3, 5, nonce=1), ctx.encrypt(1, B, 4, 3, 5, nonce=1), 4, 3, 5).export()
    torch.cuda.synchronize()
    gc.collect()
    before = torch.cuda.memory_allocated()
    ctx.use_torch_allocator()
    ca, cb = ctx.encrypt(0, A, 4, 3, 5, nonce=1), ctx.encrypt(1, B, 4, 3, 5, nonce=1)
    outs = [ctx.hegmm(ca, cb, 4, 3, 5) for _ in range(4)]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        outs.append(ctx.hegmm(ca, cb, 4, 3, 5))
    s.synchronize()
    assert torch.cuda.memory_allocated() > before
    assert all(np.array_equal(o.export(), ref) for o in outs)
    kept = outs.pop()
    del outs
    ctx.set_allocator(None, None)
    plain = ctx.hegmm(ca, cb, 4, 3, 5)
    assert np.array_equal(plain.export(), ref)
    del kept, ca, cb, plain
    gc.collect()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
    with pytest.raises(hg.HGError) as e:   # alloc without release
        hg._check(hg._lib.hg_set_allocator(ctx.ptr, hg._ALLOC_FN(lambda n, s, u: None), hg._RELEASE_FN(), None))
    assert e.value.code == hg.HG_EINVAL
