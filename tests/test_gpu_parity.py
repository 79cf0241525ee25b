"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Every comparison is on the canonical serialisation (coefficient form,
residues in [0, q_i)), element by element; the bar is bit-identity.  Results
are also decrypted and compared with brute-force matrix products."""
import json
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2405_02238_amd as hg  # noqa: E402
from oracle import bgv, hegmm as H  # noqa: E402
from oracle.ring import Params  # noqa: E402


def flat(ct):
    return H.export_d7(ct)


class Pair:
    """A library context and the oracle's key set for the same parameters and seed."""

    def __init__(self, N, t, L, alpha, seed, shapes=(), zs=(), min_blocks=1, relin=0, ks_order=0, prime_bits=50):
        self.P = Params(N, t, L, alpha, prime_bits=prime_bits)
        self.min_blocks = min_blocks
        self.relin = relin
        self.ks_order = ks_order
        self.ctx = hg.Context(N, t, L, alpha, min_blocks=min_blocks, relin=relin, ks_order=ks_order,
                              prime_bits=prime_bits)
        self.ctx.keygen(seed, shapes)
        if zs:
            self.ctx.keygen_rotations(zs)
        gal = H.galois_elements(self.P, shapes, min_blocks=min_blocks) + [self.P.galois(z) for z in zs]
        self.ks = bgv.KeySet(self.P, seed, gal)
        self.masks = H.MaskCache(self.P)


@pytest.fixture(scope="module")
def tiny():
    c = workloads.TINY
    return Pair(c.N, c.t, c.L, c.alpha, c.seed, shapes=[(4, 3, 5), (2, 5, 7), (5, 4, 2), (3, 11, 6), (7, 7, 7)],
                zs=[1, 3, -2, 17])


def test_primes(tiny):
    assert tiny.ctx.primes() == tiny.P.ext


def test_encrypt_bits(tiny):
    rng = np.random.default_rng(1)
    v = rng.integers(0, tiny.P.t, tiny.P.S)
    got = tiny.ctx.encrypt_slots(v, nonce=9).export()
    want = flat(bgv.encrypt_slots(tiny.ks, [int(x) for x in v], role=2, block=0, nonce=9))
    assert got.shape == want.shape
    assert np.array_equal(got, want)


def test_export_import_roundtrip(tiny):
    v = np.arange(tiny.P.S) % tiny.P.t
    ct = tiny.ctx.encrypt_slots(v, nonce=3)
    w = ct.export()
    back = tiny.ctx.import_ct(w, 1, 2)
    assert np.array_equal(back.export(), w)
    assert np.array_equal(tiny.ctx.decrypt_slots(back), v)


@pytest.mark.parametrize("z", [1, 3, -2, 17])
def test_rotate_bits(tiny, z):
    rng = np.random.default_rng(10 + z)
    v = [int(x) for x in rng.integers(0, tiny.P.t, tiny.P.S)]
    ct = tiny.ctx.encrypt_slots(v, nonce=20 + z)
    got = tiny.ctx.rotate(ct, z).export()
    oc = bgv.encrypt_slots(tiny.ks, v, role=2, block=0, nonce=20 + z)
    want = flat(bgv.rotate(tiny.P, tiny.ks, oc, z))
    assert np.array_equal(got, want)
    dec = tiny.ctx.decrypt_slots(tiny.ctx.import_ct(got, 1, 2))
    assert list(dec) == [v[(s + z) % tiny.P.S] for s in range(tiny.P.S)]


def test_mul_bits(tiny):
    rng = np.random.default_rng(5)
    a = [int(x) for x in rng.integers(0, tiny.P.t, tiny.P.S)]
    b = [int(x) for x in rng.integers(0, tiny.P.t, tiny.P.S)]
    ca, cb = tiny.ctx.encrypt_slots(a, nonce=1), tiny.ctx.encrypt_slots(b, nonce=2)
    got = tiny.ctx.mul(ca, cb).export()
    oa = bgv.encrypt_slots(tiny.ks, a, role=2, block=0, nonce=1)
    ob = bgv.encrypt_slots(tiny.ks, b, role=2, block=0, nonce=2)
    want = flat(bgv.he_mult(tiny.P, tiny.ks, oa, ob))
    assert np.array_equal(got, want)


def run_pair(pair, m, l, n, A, B, nonce):
    ctx, P, ks = pair.ctx, pair.P, pair.ks
    ca = ctx.encrypt(0, A, m, l, n, nonce=nonce)
    cb = ctx.encrypt(1, B, m, l, n, nonce=nonce)
    pl = H.plan(m, l, n, P.S, min_blocks=pair.min_blocks)
    ox = H.encrypt_operand(ks, pl, 0, A, B, nonce)
    oy = H.encrypt_operand(ks, pl, 1, A, B, nonce)
    # operands: bit-identical packing + encryption
    left, right = (cb, ca) if pl.transposed else (ca, cb)
    assert np.array_equal(left.export(), np.concatenate([flat(c) for c in ox]))
    assert np.array_equal(right.export(), np.concatenate([flat(c) for c in oy]))
    cc = ctx.hegmm(ca, cb, m, l, n)
    got = cc.export()
    want = flat(H.hegmm(ks, pl, ox, oy, pair.masks, eager=pair.relin == 1, ks_order=pair.ks_order))
    assert np.array_equal(got, want), (m, l, n)
    C = ctx.decrypt(cc, m, l, n)
    assert np.array_equal(C, workloads.plain_matmul_mod(A, B, P.t))


def test_hegmm_tiny_config(tiny):
    A, B = workloads.tiny_operands()
    run_pair(tiny, 4, 3, 5, A, B, nonce=1)


@pytest.mark.parametrize("shape", [(2, 5, 7), (5, 4, 2), (3, 11, 6), (7, 7, 7)],
                         ids=["dupA-fold", "transposed", "blocked", "square"])
def test_hegmm_shapes(tiny, shape):
    m, l, n = shape
    rng = np.random.default_rng(sum(shape))
    A = rng.integers(-8, 9, size=(m, l))
    B = rng.integers(-8, 9, size=(l, n))
    run_pair(tiny, m, l, n, A, B, nonce=7)


def test_hegmm_degenerate_shapes():
    """Shapes at the method's edges, each bit-identical to the oracle and
    decrypting to A.B mod t: 1x1x1 and an inner dimension of 1 (one loop
    trip, no rotation at all: only the relinearisation key switch), a single
    row of A (six stacked copies of A and a fold of five rotations), a single
    column of B (the transposed orientation), and a product that fills the
    512 slots of the ring exactly (M W = 16 x 32)."""
    c = workloads.TINY
    shapes = [(1, 1, 1), (1, 5, 1), (1, 1, 6), (6, 1, 1), (3, 1, 4), (1, 6, 4), (4, 6, 1), (16, 16, 32)]
    pair = Pair(c.N, c.t, c.L, c.alpha, c.seed + 5, shapes=shapes)
    assert pair.ctx.plan_info(1, 1, 1)["rotations"] == 0
    rng = np.random.default_rng(77)
    ops = []
    for i, (m, l, n) in enumerate(shapes):
        A = rng.integers(-8, 9, size=(m, l))
        B = rng.integers(-8, 9, size=(l, n))
        run_pair(pair, m, l, n, A, B, nonce=60 + i)
        ops.append((pair.ctx.encrypt(0, A, m, l, n, nonce=60 + i), pair.ctx.encrypt(1, B, m, l, n, nonce=60 + i)))
    # the same products in one batch (shared launches): each result as alone
    alone = [pair.ctx.hegmm(a, b, *s).export() for (a, b), s in zip(ops, shapes)]
    batch = pair.ctx.hegmm_batch([a for a, _ in ops], [b for _, b in ops], shapes)
    for s, got, want in zip(shapes, batch, alone):
        assert np.array_equal(got.export(), want), s


@pytest.mark.parametrize("min_blocks", [2, 3])
def test_hegmm_forced_blocks(min_blocks):
    """The blockwise product (inner dimension split into at least k blocks,
    one accumulator) forced on shapes that fit whole: bits equal the oracle's
    with the same plan, and the result decrypts to A.B mod t."""
    c = workloads.TINY
    shapes = [(4, 3, 5), (2, 5, 7), (5, 4, 2), (7, 7, 7)]
    pair = Pair(c.N, c.t, c.L, c.alpha, c.seed, shapes=shapes, min_blocks=min_blocks)
    rng = np.random.default_rng(60 + min_blocks)
    for i, (m, l, n) in enumerate(shapes):
        A = rng.integers(-8, 9, size=(m, l))
        B = rng.integers(-8, 9, size=(l, n))
        assert pair.ctx.plan_info(m, l, n)["nb"] == min(min_blocks, l)
        run_pair(pair, m, l, n, A, B, nonce=11 + i)


def test_hegmm_alpha2():
    pair = Pair(1024, 12289, 4, 2, 99, shapes=[(3, 7, 5), (6, 4, 9)])
    rng = np.random.default_rng(3)
    for (m, l, n) in [(3, 7, 5), (6, 4, 9)]:
        A = rng.integers(-8, 9, size=(m, l))
        B = rng.integers(-8, 9, size=(l, n))
        run_pair(pair, m, l, n, A, B, nonce=5)


@pytest.mark.parametrize("N", [4096, 8192])
@pytest.mark.parametrize("radix", [8, 16])
def test_hegmm_row_radix(N, radix):
    """Both radices of the 4096- and 8192-point row transforms (radix 8 is
    the built-in choice, radix 16 the tuning alternative): bits equal the
    oracle's, and the result decrypts to A.B mod t."""
    shapes = [(6, 5, 9)]
    pair = Pair(N, 65537, 3, 1, 70 + N // 4096, shapes=shapes)
    rng = np.random.default_rng(N + radix)
    A = rng.integers(-8, 9, size=(6, 5))
    B = rng.integers(-8, 9, size=(5, 9))
    pair.ctx.tune("ntt_radix", radix)
    try:
        run_pair(pair, 6, 5, 9, A, B, nonce=3)
    finally:
        pair.ctx.tune("ntt_radix", 0)


@pytest.mark.parametrize("alpha", [1, 2])
def test_eager_relin_shapes(alpha):
    """Eager relinearisation (every loop product relinearised on its own):
    bits equal the oracle's eager mode on fold, transposed, blocked and
    forced-block shapes, and each result decrypts to A.B mod t."""
    c = workloads.TINY
    L = c.L if alpha == 1 else 4
    shapes = [(4, 3, 5), (2, 5, 7), (5, 4, 2), (3, 11, 6), (1, 4, 3)]
    pair = Pair(c.N, c.t, L, alpha, c.seed + alpha, shapes=shapes, relin=1)
    rng = np.random.default_rng(90 + alpha)
    for i, (m, l, n) in enumerate(shapes):
        A = rng.integers(-8, 9, size=(m, l))
        B = rng.integers(-8, 9, size=(l, n))
        run_pair(pair, m, l, n, A, B, nonce=20 + i)
    forced = Pair(c.N, c.t, c.L, 1, c.seed, shapes=[(5, 4, 2)], min_blocks=2, relin=1)
    A = rng.integers(-8, 9, size=(5, 4))
    B = rng.integers(-8, 9, size=(4, 2))
    run_pair(forced, 5, 4, 2, A, B, nonce=30)


def test_eager_relin_batch_and_graph():
    """Eager relinearisation inside a batch and a recorded graph: every
    result is the bit pattern of the same product run alone; with one loop
    product (K = 1) eager and lazy contexts give the same bits."""
    c = workloads.TINY
    shapes = [(4, 3, 5), (2, 5, 7), (5, 4, 2), (1, 4, 3)]
    ctx = hg.Context(c.N, c.t, c.L, c.alpha, relin=1)
    lazy = hg.Context(c.N, c.t, c.L, c.alpha)
    for x in (ctx, lazy):
        x.keygen(c.seed, shapes)
    rng = np.random.default_rng(95)
    mats = [(rng.integers(-8, 9, size=(m, l)), rng.integers(-8, 9, size=(l, n))) for (m, l, n) in shapes]
    As = [ctx.encrypt(0, A, *s, nonce=40 + i) for i, (s, (A, B)) in enumerate(zip(shapes, mats))]
    Bs = [ctx.encrypt(1, B, *s, nonce=40 + i) for i, (s, (A, B)) in enumerate(zip(shapes, mats))]
    alone = [ctx.hegmm(a, b, *s).export() for a, b, s in zip(As, Bs, shapes)]
    got = ctx.hegmm_batch(As, Bs, shapes)
    for i, s in enumerate(shapes):
        assert np.array_equal(got[i].export(), alone[i]), s
        assert np.array_equal(ctx.decrypt(got[i], *s), workloads.plain_matmul_mod(*mats[i], c.t)), s
    g = ctx.record_batch(As, Bs, shapes)
    zero = np.zeros_like(alone[0])
    for rep in range(3):
        for o in g.outputs:
            ctx.load_ct(o, zero)
        ctx.hegmm(As[rep], Bs[rep], *shapes[rep])     # eager work between replays
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        for i, s in enumerate(shapes):
            assert np.array_equal(g.outputs[i].export(), alone[i]), (rep, s)
    g.close()
    m, l, n = shapes[3]
    la = lazy.encrypt(0, mats[3][0], m, l, n, nonce=43)
    lb = lazy.encrypt(1, mats[3][1], m, l, n, nonce=43)
    assert np.array_equal(lazy.hegmm(la, lb, m, l, n).export(), alone[3])


def test_eager_relin_headline_full_size():
    """64x32x48 at N = 8192 with eager relinearisation (32 key switches of
    the tensor products instead of one): the whole output against the oracle."""
    c = workloads.HEADLINE
    pair = Pair(c.N, c.t, c.L, c.alpha, c.seed, shapes=[(64, 32, 48)], relin=1)
    A, B = workloads.headline_operands()
    run_pair(pair, 64, 32, 48, A, B, nonce=1)


def test_mod_switch_result(tiny):
    """Modulus switching of a product result by one and two primes: bits equal
    the oracle's switching of the oracle's (bit-identical) result, the export
    shrinks to 2 (L - drop) N words, and the result decrypts to A.B mod t."""
    ctx, P, ks = tiny.ctx, tiny.P, tiny.ks
    m, l, n = 4, 3, 5
    A, B = workloads.tiny_operands()
    pl = H.plan(m, l, n, P.S)
    ox = H.encrypt_operand(ks, pl, 0, A, B, 1)
    oy = H.encrypt_operand(ks, pl, 1, A, B, 1)
    R = H.hegmm(ks, pl, ox, oy, tiny.masks)
    cc = ctx.hegmm(ctx.encrypt(0, A, m, l, n, nonce=1), ctx.encrypt(1, B, m, l, n, nonce=1), m, l, n)
    assert np.array_equal(cc.export(), flat(R))
    for drop in range(1, P.L):
        sw = ctx.mod_switch(cc, drop)
        got = sw.export()
        assert got.size == 2 * (P.L - drop) * P.N
        assert np.array_equal(got, flat(bgv.mod_switch(P, R, drop))), drop
        assert np.array_equal(ctx.decrypt(sw, m, l, n), workloads.plain_matmul_mod(A, B, P.t)), drop
    one = ctx.mod_switch(cc, 1)
    with pytest.raises(hg.HGError):
        ctx.mod_switch(cc, P.L)
    with pytest.raises(hg.HGError):
        ctx.mod_switch(cc, 0)
    with pytest.raises(hg.HGError):
        ctx.mod_switch(one, P.L - 1)
    with pytest.raises(hg.HGError):
        ctx.rotate(one, 1)
    with pytest.raises(hg.HGError):
        ctx.hegmm(one, cc, m, l, n)


@pytest.mark.parametrize("cfg", ["serving", "large"])
def test_mod_switch_fresh_large_rings(cfg):
    """Modulus switching at N = 16384 (6 + 2 primes, one-workgroup rows) and
    N = 32768 (8 + 2 primes, two-pass transforms) on fresh encryptions: bits
    equal the oracle's switching of the same (bit-identical) encryption, and
    the slots decrypt unchanged."""
    c = workloads.CONFIGS[cfg]
    P = Params(c.N, c.t, c.L, c.alpha)
    ctx = hg.Context(c.N, c.t, c.L, c.alpha)
    ctx.keygen(c.seed, [])
    ks = bgv.KeySet(P, c.seed, [], relin=False)
    rng = np.random.default_rng(c.N)
    v = rng.integers(0, P.t, P.S)
    ct = ctx.encrypt_slots(v, nonce=5)
    ref = bgv.encrypt_slots(ks, [int(x) for x in v], role=2, block=0, nonce=5)
    assert np.array_equal(ct.export(), flat(ref))
    for drop in (1, 3):
        sw = ctx.mod_switch(ct, drop)
        assert np.array_equal(sw.export(), flat(bgv.mod_switch(P, ref, drop))), drop
        assert np.array_equal(ctx.decrypt_slots(sw), v.astype(np.int64)), drop


@pytest.mark.parametrize("alpha", [1, 2])
def test_paper_order_shapes(alpha):
    """Linear transforms in the paper's primitive order (ks_order 1: one
    complete HE-Rot per diagonal, then HE-CMult, then HE-Add; Section III-B-1,
    Eq. (lintrans)): bits equal the oracle's paper-order composition on the
    C1 shape and the fold, transposed, blocked and square plans, and every
    result decrypts to A.B mod t.  The deferred order gives other bits on
    shapes with masked diagonals, the same decryption."""
    c = workloads.TINY
    L = c.L if alpha == 1 else 4
    shapes = [(4, 3, 5), (2, 5, 7), (5, 4, 2), (3, 11, 6), (7, 7, 7)]
    pair = Pair(c.N, c.t, L, alpha, c.seed + 7 * alpha, shapes=shapes, ks_order=1)
    rng = np.random.default_rng(120 + alpha)
    for i, (m, l, n) in enumerate(shapes):
        A = rng.integers(-8, 9, size=(m, l))
        B = rng.integers(-8, 9, size=(l, n))
        run_pair(pair, m, l, n, A, B, nonce=50 + i)
    m, l, n = shapes[0]
    A, B = workloads.tiny_operands()
    deferred = hg.Context(c.N, c.t, L, alpha)
    deferred.keygen(c.seed + 7 * alpha, [(m, l, n)])
    cd = deferred.hegmm(deferred.encrypt(0, A, m, l, n, nonce=1), deferred.encrypt(1, B, m, l, n, nonce=1), m, l, n)
    cp = pair.ctx.hegmm(pair.ctx.encrypt(0, A, m, l, n, nonce=1), pair.ctx.encrypt(1, B, m, l, n, nonce=1), m, l, n)
    assert not np.array_equal(cd.export(), cp.export())
    assert np.array_equal(deferred.decrypt(cd, m, l, n), pair.ctx.decrypt(cp, m, l, n))


def test_paper_order_variants():
    """The paper's primitive order under eager relinearisation, forced inner
    blocks, and Algorithm 1 with sigma / tau on the ciphertexts (method 3):
    bits equal the oracle's, results decrypt to A.B mod t."""
    c = workloads.TINY
    rng = np.random.default_rng(131)
    shapes = [(4, 3, 5), (2, 5, 7), (5, 4, 2)]
    eager = Pair(c.N, c.t, c.L, c.alpha, c.seed, shapes=shapes, relin=1, ks_order=1)
    for i, (m, l, n) in enumerate(shapes):
        run_pair(eager, m, l, n, rng.integers(-8, 9, size=(m, l)), rng.integers(-8, 9, size=(l, n)), nonce=60 + i)
    forced = Pair(c.N, c.t, c.L, c.alpha, c.seed, shapes=[(5, 4, 2), (4, 3, 5)], min_blocks=2, ks_order=1)
    for i, (m, l, n) in enumerate([(5, 4, 2), (4, 3, 5)]):
        run_pair(forced, m, l, n, rng.integers(-8, 9, size=(m, l)), rng.integers(-8, 9, size=(l, n)), nonce=70 + i)
    P = Params(c.N, c.t, c.L, c.alpha)
    ctx = hg.Context(c.N, c.t, c.L, c.alpha, method=3, ks_order=1)
    for i, (m, l, n) in enumerate([(3, 4, 5), (5, 3, 4)]):
        ctx.keygen(c.seed, [(m, l, n)])
        pl = H.plan(m, l, n, P.S, method=3)
        ks = bgv.KeySet(P, c.seed, H.galois_elements(P, [(m, l, n)], method=3))
        A = rng.integers(-8, 9, size=(m, l))
        B = rng.integers(-8, 9, size=(l, n))
        cc = ctx.hegmm(ctx.encrypt(0, A, m, l, n, nonce=80 + i), ctx.encrypt(1, B, m, l, n, nonce=80 + i), m, l, n)
        ox = H.encrypt_operand(ks, pl, 0, A, B, 80 + i)
        oy = H.encrypt_operand(ks, pl, 1, A, B, 80 + i)
        assert np.array_equal(cc.export(), flat(H.hegmm(ks, pl, ox, oy, ks_order=1))), (m, l, n)
        assert np.array_equal(ctx.decrypt(cc, m, l, n), workloads.plain_matmul_mod(A, B, c.t))


def test_paper_order_headline_full_size():
    """64x32x48 at N = 8192 in the paper's primitive order (124 rotations,
    each divided by P on its own, masks after): the whole output against the
    oracle's paper-order composition."""
    c = workloads.HEADLINE
    pair = Pair(c.N, c.t, c.L, c.alpha, c.seed, shapes=[(64, 32, 48)], ks_order=1)
    A, B = workloads.headline_operands()
    run_pair(pair, 64, 32, 48, A, B, nonce=1)


def test_prime_bits_honoured():
    """Primes below 2^40 instead of 2^50 (hg_params.prime_bits): the library's
    primes are the oracle's, and a product is bit-identical to the oracle's
    with those primes."""
    c = workloads.TINY
    pair = Pair(c.N, c.t, c.L, c.alpha, c.seed, shapes=[(4, 3, 5), (2, 5, 7)], prime_bits=40)
    assert pair.ctx.primes() == pair.P.ext
    assert all(p < 2 ** 40 for p in pair.P.ext)
    A, B = workloads.tiny_operands()
    run_pair(pair, 4, 3, 5, A, B, nonce=1)
    rng = np.random.default_rng(140)
    run_pair(pair, 2, 5, 7, rng.integers(-8, 9, size=(2, 5)), rng.integers(-8, 9, size=(5, 7)), nonce=2)


def test_hegmm_twelve_digits():
    """L = 12 ciphertext primes with one-prime digits: the key-switch inner
    products add 12 digit products, reduced after the 8th (the longest sums
    the library builds); bits equal the oracle's, the result decrypts."""
    c = workloads.TINY
    pair = Pair(c.N, c.t, 12, 1, c.seed, shapes=[(4, 3, 5), (2, 5, 7)])
    A, B = workloads.tiny_operands()
    run_pair(pair, 4, 3, 5, A, B, nonce=1)
    rng = np.random.default_rng(150)
    run_pair(pair, 2, 5, 7, rng.integers(-8, 9, size=(2, 5)), rng.integers(-8, 9, size=(5, 7)), nonce=2)


def test_hegmm_headline_full_size():
    """64x32x48 at N = 8192: the whole output ciphertext against the oracle."""
    c = workloads.HEADLINE
    pair = Pair(c.N, c.t, c.L, c.alpha, c.seed, shapes=[(64, 32, 48)])
    A, B = workloads.headline_operands()
    run_pair(pair, 64, 32, 48, A, B, nonce=1)


def test_batch_matches_alone_and_oracle(tiny):
    """Products batched into shared launches give the same bits as alone, and
    as the oracle (repeated shapes share key groups in the batch)."""
    shapes = [(2, 5, 7), (5, 4, 2), (3, 11, 6), (7, 7, 7), (4, 3, 5), (2, 5, 7), (7, 7, 7)]
    rng = np.random.default_rng(21)
    mats = [(rng.integers(-8, 9, size=(m, l)), rng.integers(-8, 9, size=(l, n))) for (m, l, n) in shapes]
    ctx = tiny.ctx
    As = [ctx.encrypt(0, A, *s, nonce=100 + i) for i, (s, (A, B)) in enumerate(zip(shapes, mats))]
    Bs = [ctx.encrypt(1, B, *s, nonce=100 + i) for i, (s, (A, B)) in enumerate(zip(shapes, mats))]
    outs = ctx.hegmm_batch(As, Bs, shapes)
    for i, (s, (A, B)) in enumerate(zip(shapes, mats)):
        alone = ctx.hegmm(As[i], Bs[i], *s)
        assert np.array_equal(outs[i].export(), alone.export()), s
        assert np.array_equal(ctx.decrypt(outs[i], *s), workloads.plain_matmul_mod(A, B, tiny.P.t)), s
    for i in (0, 2, 6):
        m, l, n = shapes[i]
        A, B = mats[i]
        pl = H.plan(m, l, n, tiny.P.S)
        ox = H.encrypt_operand(tiny.ks, pl, 0, A, B, 100 + i)
        oy = H.encrypt_operand(tiny.ks, pl, 1, A, B, 100 + i)
        want = flat(H.hegmm(tiny.ks, pl, ox, oy, tiny.masks))
        assert np.array_equal(outs[i].export(), want), shapes[i]


def _golden(name):
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"{name}_oracle.json")
    assert os.path.exists(path), f"{path} missing: run tests/golden/make_workload_golden.py"
    return json.load(open(path))


def test_batched_workload_every_result():
    """The 256-request mixed-shape batch at N = 8192 (shapes uniform over
    {8, ..., 64}^3, inner blocking and folds included): every result equals
    the oracle's bit for bit (SHA-256 of its canonical words, written by the
    oracle alone) and decrypts to A.B mod t."""
    c = workloads.BATCHED
    reqs = workloads.batched_requests(256)
    g = _golden("batched")
    assert g["seed"] == c.seed and len(g["requests"]) == len(reqs)
    shapes = [(m, l, n) for (m, l, n, _, _) in reqs]
    assert [tuple(r["shape"]) for r in g["requests"]] == shapes
    ctx = hg.Context(c.N, c.t, c.L, c.alpha)
    ctx.keygen(c.seed, shapes)
    As = [ctx.encrypt(0, A, m, l, n, nonce=i) for i, (m, l, n, A, B) in enumerate(reqs)]
    Bs = [ctx.encrypt(1, B, m, l, n, nonce=i) for i, (m, l, n, A, B) in enumerate(reqs)]
    outs = ctx.hegmm_batch(As, Bs, shapes)
    P = Params(c.N, c.t, c.L, c.alpha)
    kinds = {"blocked": 0, "folded": 0, "transposed": 0}
    for i, (m, l, n, A, B) in enumerate(reqs):
        assert _sha(outs[i].export()) == g["requests"][i]["result_sha256"], (i, m, l, n)
        assert np.array_equal(ctx.decrypt(outs[i], m, l, n), workloads.plain_matmul_mod(A, B, c.t)), (i, m, l, n)
        pl = H.plan(m, l, n, P.S)
        kinds["blocked"] += pl.nb > 1
        kinds["folded"] += pl.d > 1
        kinds["transposed"] += bool(pl.transposed)
    assert all(v > 0 for v in kinds.values()), kinds


def test_serving_mix_equals_alone():
    """Continuous batching at N = 16384 (6 + 2 primes) on 64 requests: a burst
    queued while admission is held fills whole groups on both lanes at once
    (mean group > 1, two groups in flight, modelled memory within the
    budget); then the same requests arrive Poisson-timed (tenfold compressed)
    and are admitted while others run.  Every served result, in both runs,
    equals the product alone and the oracle's result bit for bit, and
    decrypts to A.B mod t."""
    from paper_2405_02238_amd import serving
    c = workloads.SERVING
    g = _golden("serving")
    reqs = workloads.serving_requests(len(g["requests"]))
    assert g["seed"] == c.seed
    assert [tuple(r["shape"]) for r in g["requests"]] == [(m, l, n) for (_, m, l, n, _, _) in reqs]
    shapes = sorted({(m, l, n) for (_, m, l, n, _, _) in reqs})
    ctx = hg.Context(c.N, c.t, c.L, c.alpha)
    ctx.keygen(c.seed, shapes)
    cts, timed = [], []
    for i, (at, m, l, n, A, B) in enumerate(reqs):
        ca, cb = ctx.encrypt(0, A, m, l, n, nonce=i), ctx.encrypt(1, B, m, l, n, nonce=i)
        cts.append((ca, cb))
        timed.append((at / 10.0, m, l, n, ca.export(), cb.export()))
    alone = [ctx.hegmm(cts[i][0], cts[i][1], *timed[i][1:4]).export() for i in range(len(reqs))]
    for i, w in enumerate(alone):
        assert _sha(w) == g["requests"][i]["result_sha256"], i
    fps = [ctx.request_footprint(m, l, n) for (_, m, l, n, _, _) in reqs]
    budget = 24 * max(fps)
    with hg.Server(ctx, max_batch=8, lanes=2, hbm_budget=budget) as srv:
        srv.pause(True)
        tickets = [srv.submit(a, b, m, l, n) for (_, m, l, n, a, b) in timed]
        assert srv.stats()["queued"] == len(reqs)
        srv.pause(False)
        burst = [srv.wait(t)[0] for t in tickets]
        st = srv.stats()
        results, lat, _ = serving.replay(srv, timed)
    assert st["done"] == len(reqs)
    assert st["mean_group"] == 8.0, st
    assert st["peak_lanes_busy"] >= 2, st
    assert st["peak_footprint"] <= budget, st
    for i, (at, m, l, n, A, B) in enumerate(reqs):
        assert np.array_equal(burst[i], alone[i]), (i, m, l, n)
        assert np.array_equal(results[i], alone[i]), (i, m, l, n)
        C = ctx.decrypt(ctx.import_ct(results[i], 1, 2), m, l, n)
        assert np.array_equal(C, workloads.plain_matmul_mod(A, B, c.t)), (i, m, l, n)


def test_tune_refused_while_served_and_per_context():
    """hg_tune, and every other call on the context but hg_server_* and
    hg_request_footprint (a product, an encryption, a decryption, a second
    server), is refused while a server owns the context; a knob set on one
    context leaves another's results (and knobs) alone."""
    c = workloads.TINY
    a = hg.Context(c.N, c.t, c.L, c.alpha)
    b = hg.Context(c.N, c.t, c.L, c.alpha)
    for x in (a, b):
        x.keygen(c.seed, [(4, 3, 5)])
    A, B = workloads.tiny_operands()
    ca, cb = a.encrypt(0, A, 4, 3, 5, nonce=1), a.encrypt(1, B, 4, 3, 5, nonce=1)
    want = a.hegmm(ca, cb, 4, 3, 5).export()
    wa, wb = ca.export(), cb.export()
    with hg.Server(a, max_batch=2, lanes=1) as srv:
        refused = [lambda: a.tune("ntt_radix", 16), lambda: a.hegmm(ca, cb, 4, 3, 5),
                   lambda: a.encrypt(0, A, 4, 3, 5, nonce=2), lambda: a.decrypt(ca, 4, 3, 5),
                   lambda: ca.export(), lambda: hg.Server(a, max_batch=2, lanes=1)]
        for call in refused:
            with pytest.raises(hg.HGError) as e:
                call()
            assert e.value.code == hg.HG_ESTATE
        assert a.request_footprint(4, 3, 5) > 0
        served, _ = srv.wait(srv.submit(wa, wb, 4, 3, 5))
        assert np.array_equal(served, want)   # the server runs on after the refusals
        b.tune("half_rows", 0)          # another context stays tunable
        srv.pause(True)
        srv.pause(False)
    a.tune("ntt_radix", 16)             # allowed again once the server is gone
    got = b.hegmm(b.encrypt(0, A, 4, 3, 5, nonce=1), b.encrypt(1, B, 4, 3, 5, nonce=1), 4, 3, 5).export()
    assert np.array_equal(got, want)


def test_serving_memory_within_model():
    """The device memory a server lane takes for an admitted group, measured
    with hipMemGetInfo (free memory before the group against the lowest free
    memory seen while it runs and after it), stays within the modelled bytes
    the server admitted it under, and those within the sum of
    hg_request_footprint over the group."""
    c = workloads.SERVING
    reqs = workloads.serving_requests(12, seed_offset=7)
    shapes = sorted({(m, l, n) for (_, m, l, n, _, _) in reqs})
    ctx = hg.Context(c.N, c.t, c.L, c.alpha)
    ctx.keygen(c.seed, shapes)
    words = []
    for i, (at, m, l, n, A, B) in enumerate(reqs):
        words.append((ctx.encrypt(0, A, m, l, n, nonce=i).export(), ctx.encrypt(1, B, m, l, n, nonce=i).export()))
    model = sum(ctx.request_footprint(m, l, n) for (_, m, l, n, _, _) in reqs)
    with hg.Server(ctx, max_batch=len(reqs), lanes=1, hbm_budget=0) as srv:
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        srv.pause(True)
        tickets = [srv.submit(a, b, m, l, n) for (a, b), (_, m, l, n, _, _) in zip(words, reqs)]
        srv.pause(False)
        low = free0
        while srv.stats()["done"] < len(reqs):
            low = min(low, torch.cuda.mem_get_info()[0])
        outs = [srv.wait(t)[0] for t in tickets]
        low = min(low, torch.cuda.mem_get_info()[0])
        st = srv.stats()
    used = free0 - low
    assert st["groups"] == 1 and st["mean_group"] == len(reqs), st
    assert 0 < used <= st["peak_footprint"] <= model, (used, st["peak_footprint"], model)
    for (_, m, l, n, A, B), w in zip(reqs, outs):
        assert np.array_equal(ctx.decrypt(ctx.import_ct(w, 1, 2), m, l, n), workloads.plain_matmul_mod(A, B, c.t))


def test_serving_errors_and_budget():
    """Unkeyed shapes and malformed operands are refused at submission; a
    budget below one request still serves it alone."""
    c = workloads.TINY
    ctx = hg.Context(c.N, c.t, c.L, c.alpha)
    ctx.keygen(c.seed, [(4, 3, 5)])
    A, B = workloads.tiny_operands()
    wa = ctx.encrypt(0, A, 4, 3, 5, nonce=3).export()
    wb = ctx.encrypt(1, B, 4, 3, 5, nonce=3).export()
    with hg.Server(ctx, max_batch=4, lanes=1, hbm_budget=1) as srv:
        with pytest.raises(hg.HGError) as e:
            srv.submit(wa, wb, 5, 3, 4)
        assert e.value.code == hg.HG_ENOKEY
        with pytest.raises(hg.HGError) as e:
            srv.submit(wa[:-1], wb, 4, 3, 5)
        assert e.value.code == hg.HG_EINVAL
        bad = wa.copy()
        bad[0] = np.uint64(2 ** 63)
        with pytest.raises(hg.HGError):
            srv.submit(bad, wb, 4, 3, 5)
        tickets = [srv.submit(wa, wb, 4, 3, 5) for _ in range(3)]
        outs = [srv.wait(t)[0] for t in tickets]
        assert srv.stats()["mean_group"] == 1.0
    for o in outs:
        assert np.array_equal(ctx.decrypt(ctx.import_ct(o, 1, 2), 4, 3, 5),
                              workloads.plain_matmul_mod(A, B, c.t))


@pytest.mark.parametrize("variant", [{"relin": 1}, {"method": 3}, {"method": 3, "relin": 1}])
def test_serving_variants_equal_alone(variant):
    """The request loop serves contexts of every variant (eager
    relinearisation, Algorithm 1 with cloud-side sigma/tau): each served
    result is the bit pattern of the same product run alone."""
    c = workloads.TINY
    ctx = hg.Context(c.N, c.t, c.L, c.alpha, **variant)
    shapes = [(4, 3, 5), (2, 5, 3), (3, 3, 3)]
    ctx.keygen(c.seed, shapes)
    rng = np.random.default_rng(31)
    reqs = []
    for i, (m, l, n) in enumerate(shapes * 2):
        A = rng.integers(-8, 9, size=(m, l))
        B = rng.integers(-8, 9, size=(l, n))
        ca, cb = ctx.encrypt(0, A, m, l, n, nonce=50 + i), ctx.encrypt(1, B, m, l, n, nonce=50 + i)
        reqs.append((m, l, n, A, B, ca, cb))
    alone = [ctx.hegmm(ca, cb, m, l, n).export() for (m, l, n, A, B, ca, cb) in reqs]
    words = [(ca.export(), cb.export()) for (m, l, n, A, B, ca, cb) in reqs]
    with hg.Server(ctx, max_batch=4, lanes=2) as srv:
        tickets = [srv.submit(wa, wb, m, l, n) for (wa, wb), (m, l, n, A, B, ca, cb) in zip(words, reqs)]
        outs = [srv.wait(t)[0] for t in tickets]
    for (m, l, n, A, B, ca, cb), o, w in zip(reqs, outs, alone):
        assert np.array_equal(o, w), (m, l, n)
        assert np.array_equal(ctx.decrypt(ctx.import_ct(o, 1, 2), m, l, n), workloads.plain_matmul_mod(A, B, c.t))


def _sha(words):
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(words, dtype="<u8").tobytes()).hexdigest()


def _offsets(sizes):
    return [int(x) for x in np.cumsum((0,) + tuple(sizes))[:-1]]


@pytest.mark.parametrize("part", ["P1", "P2"])
def test_blocked_100x100(part):
    """A 100x100 by 100x100 product whose result does not fit one ciphertext
    (10000 > 4096 slots), through the ABI as an output-blocked product with
    the paper's partitions (Section IV-D, Table IV): hg_set_partition, one
    hg_encrypt per operand, one hg_hegmm (the four block products in one
    batch, each splitting its inner dimension itself), one hg_decrypt that
    places the blocks.  C == A.B mod t; every block's ciphertext equals the
    oracle's product of that block (nonce 65536 nonce + k) bit for bit.  For
    P1 the paper's own split of the inner dimension too (eight 50x50x50
    products, partial results added with HE-Add) gives the same C."""
    c = workloads.HEADLINE
    D = workloads.BLOCKED_DIM
    A, B = workloads.blocked_operands()
    rows, cols = workloads.PARTITIONS[part]
    r0, c0 = _offsets(rows), _offsets(cols)
    grid = [(i, j) for i in range(len(rows)) for j in range(len(cols))]
    shapes = [(rows[i], D, cols[j]) for (i, j) in grid]
    extra = [(50, 50, 50)] if part == "P1" else []
    pair = Pair(c.N, c.t, c.L, c.alpha, c.seed, shapes=shapes + extra)
    ctx = pair.ctx
    ctx.set_partition(D, D, D, rows, cols)
    assert ctx.partition(D, D, D) == (list(rows), list(cols))
    ctx.keygen(c.seed, [(D, D, D)])
    nonce = 20
    ca, cb = ctx.encrypt(0, A, D, D, D, nonce=nonce), ctx.encrypt(1, B, D, D, D, nonce=nonce)
    out = ctx.hegmm(ca, cb, D, D, D)
    C = ctx.decrypt(out, D, D, D)
    assert np.array_equal(C, workloads.plain_matmul_mod(A, B, c.t))
    words = out.export()
    per = 2 * c.L * c.N
    assert words.size == len(grid) * per
    assert np.array_equal(ctx.decrypt(ctx.import_ct(words, len(grid), 2), D, D, D), C)
    for k, (i, j) in enumerate(grid):
        m, l, n = shapes[k]
        pl = H.plan(m, l, n, pair.P.S)
        assert pl.nb > 1
        Ab, Bb = A[r0[i]:r0[i] + m, :], B[:, c0[j]:c0[j] + n]
        ox = H.encrypt_operand(pair.ks, pl, 0, Ab, Bb, nonce * 65536 + k)
        oy = H.encrypt_operand(pair.ks, pl, 1, Ab, Bb, nonce * 65536 + k)
        assert np.array_equal(words[k * per:(k + 1) * per], flat(H.hegmm(pair.ks, pl, ox, oy, pair.masks))), k
    if part == "P1":
        # inner dimension split as well: C_ij = A_i1 B_1j + A_i2 B_2j
        k0 = _offsets((50, 50))
        s = (50, 50, 50)
        pa, pb = [], []
        for (i, j) in grid:
            for h in range(2):
                pa.append(ctx.encrypt(0, A[r0[i]:r0[i] + 50, k0[h]:k0[h] + 50], *s, nonce=40 + len(pa)))
                pb.append(ctx.encrypt(1, B[k0[h]:k0[h] + 50, c0[j]:c0[j] + 50], *s, nonce=40 + len(pb)))
        prods = ctx.hegmm_batch(pa, pb, [s] * len(pa))
        for g, (i, j) in enumerate(grid):
            blk = ctx.add(prods[2 * g], prods[2 * g + 1])
            assert np.array_equal(ctx.decrypt(blk, *s), C[r0[i]:r0[i] + 50, c0[j]:c0[j] + 50])


def test_blocked_automatic_partition():
    """Shapes whose result exceeds the 512 slots of N = 1024 get the fewest
    near-equal output blocks on their own (and a shape that fits gets none);
    every block equals the oracle's product bit for bit, C == A.B mod t, and
    a batch mixing blocked and plain products gives the same bits."""
    c = workloads.TINY
    P = Params(c.N, c.t, c.L, c.alpha)
    ctx = hg.Context(c.N, c.t, c.L, c.alpha)
    shapes = [(30, 7, 30), (40, 3, 17), (4, 3, 5)]
    parts = [ctx.partition(*s) for s in shapes]
    assert parts[2] == ([4], [5])
    for (m, l, n), (rows, cols) in zip(shapes[:2], parts[:2]):
        assert sum(rows) == m and sum(cols) == n and len(rows) * len(cols) >= 2
        assert max(rows) - min(rows) <= 1 and max(cols) - min(cols) <= 1
    ctx.keygen(c.seed, shapes)
    rng = np.random.default_rng(170)
    mats = [(rng.integers(-8, 9, size=(m, l)), rng.integers(-8, 9, size=(l, n))) for (m, l, n) in shapes]
    As = [ctx.encrypt(0, A, *s, nonce=5 + i) for i, (s, (A, B)) in enumerate(zip(shapes, mats))]
    Bs = [ctx.encrypt(1, B, *s, nonce=5 + i) for i, (s, (A, B)) in enumerate(zip(shapes, mats))]
    outs = ctx.hegmm_batch(As, Bs, shapes)
    per = 2 * c.L * c.N
    for q, ((m, l, n), (A, B), (rows, cols)) in enumerate(zip(shapes, mats, parts)):
        assert np.array_equal(ctx.decrypt(outs[q], m, l, n), workloads.plain_matmul_mod(A, B, c.t)), (m, l, n)
        alone = ctx.hegmm(As[q], Bs[q], m, l, n).export()
        words = outs[q].export()
        assert np.array_equal(words, alone)
        if len(rows) * len(cols) == 1:
            continue
        blocks = [(mi, nj, ri, cj) for ri, mi in zip(_offsets(rows), rows) for cj, nj in zip(_offsets(cols), cols)]
        ks = bgv.KeySet(P, c.seed, H.galois_elements(P, [(mi, l, nj) for (mi, nj, _, _) in blocks]))
        for k, (mi, nj, ri, cj) in enumerate(blocks):
            pl = H.plan(mi, l, nj, P.S)
            Ab, Bb = A[ri:ri + mi, :], B[:, cj:cj + nj]
            ox = H.encrypt_operand(ks, pl, 0, Ab, Bb, (5 + q) * 65536 + k)
            oy = H.encrypt_operand(ks, pl, 1, Ab, Bb, (5 + q) * 65536 + k)
            assert np.array_equal(words[k * per:(k + 1) * per], flat(H.hegmm(ks, pl, ox, oy))), ((m, l, n), k)
    with pytest.raises(hg.HGError):
        ctx.set_partition(4, 3, 5, [2, 2], [5])     # planned already as one product
    with pytest.raises(hg.HGError):
        ctx.set_partition(64, 3, 64, [60, 4], [64])  # a block of 60 x 64 results does not fit


def test_large_forced_two_blocks():
    """The large configuration's blockwise run: 128x96x128 at N = 32768 with
    the inner dimension forced into two blocks of 48 (two ciphertexts per
    operand, one accumulator); its bits differ from the one-block product by
    design, its decryption must not."""
    c = workloads.LARGE
    m, l, n = 128, 96, 128
    A, B = workloads.large_operands()
    ctx = hg.Context(c.N, c.t, c.L, c.alpha, min_blocks=2)
    info = ctx.plan_info(m, l, n)
    assert (info["nb"], info["lb"]) == (2, 48)
    ctx.keygen(c.seed, [(m, l, n)])
    ca = ctx.encrypt(0, A, m, l, n, nonce=2)
    cb = ctx.encrypt(1, B, m, l, n, nonce=2)
    assert ca.export().size == 2 * 2 * c.L * c.N
    cc = ctx.hegmm(ca, cb, m, l, n)
    assert np.array_equal(ctx.decrypt(cc, m, l, n), workloads.plain_matmul_mod(A, B, c.t))


def test_large_operands_and_product():
    """128x96x128 at N = 32768 (8 + 2 primes, two-pass transforms): packed
    operands bit-identical to the oracle's encryption, the product decrypts
    to A.B mod t, and (when the oracle's digest file is present) the result
    equals the oracle's bit for bit."""
    import json
    import os
    c = workloads.LARGE
    m, l, n = 128, 96, 128
    A, B = workloads.large_operands()
    ctx = hg.Context(c.N, c.t, c.L, c.alpha)
    ctx.keygen(c.seed, [(m, l, n)])
    ca = ctx.encrypt(0, A, m, l, n, nonce=1)
    cb = ctx.encrypt(1, B, m, l, n, nonce=1)
    P = Params(c.N, c.t, c.L, c.alpha)
    ks = bgv.KeySet(P, c.seed, [], relin=False)
    pl = H.plan(m, l, n, P.S)
    assert not pl.transposed
    assert np.array_equal(ca.export(), np.concatenate([flat(x) for x in H.encrypt_operand(ks, pl, 0, A, B, 1)]))
    assert np.array_equal(cb.export(), np.concatenate([flat(y) for y in H.encrypt_operand(ks, pl, 1, A, B, 1)]))
    cc = ctx.hegmm(ca, cb, m, l, n)
    w = cc.export()
    assert np.array_equal(ctx.decrypt(cc, m, l, n), workloads.plain_matmul_mod(A, B, c.t))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "large_oracle.json")
    if not os.path.exists(path):
        pytest.skip("oracle digest of the large product not generated (tests/golden/make_large_golden.py)")
    g = json.load(open(path))
    assert g["nonce"] == 1 and g["seed"] == c.seed
    assert _sha(ca.export()) == g["left_operand_sha256"]
    assert w.size == g["result_words"]
    for i, v in g["result_samples"].items():
        assert int(w[int(i)]) == v, i
    assert _sha(w) == g["result_sha256"]


@pytest.mark.parametrize("alpha", [1, 2])
def test_keyed_inner_products_bit_identical(alpha):
    """The key-stationary schedule (terms grouped by key, one launch per
    round of terms) gives the same bits as the plain inner products, on a
    batch with repeated shapes, folds, transposition and blocking."""
    c = workloads.TINY
    # every shape five times, so that keys repeat (the schedule is used when
    # a pass's keys are used at least four times on average)
    shapes = [(2, 5, 7), (5, 4, 2), (3, 11, 6), (4, 3, 5), (7, 7, 7), (2, 9, 3)] * 5
    ctx = hg.Context(c.N, c.t, 4 if alpha == 2 else c.L, alpha)
    ctx.keygen(c.seed, shapes)
    rng = np.random.default_rng(40 + alpha)
    mats = [(rng.integers(-8, 9, size=(m, l)), rng.integers(-8, 9, size=(l, n))) for (m, l, n) in shapes]
    As = [ctx.encrypt(0, A, *s, nonce=i) for i, (s, (A, B)) in enumerate(zip(shapes, mats))]
    Bs = [ctx.encrypt(1, B, *s, nonce=i) for i, (s, (A, B)) in enumerate(zip(shapes, mats))]
    ctx.tune("ip_chunk", 0)
    plain = [o.export() for o in ctx.hegmm_batch(As, Bs, shapes)]
    for chunk in (1, 3, 64):
        ctx.tune("ip_chunk", chunk)
        got = ctx.hegmm_batch(As, Bs, shapes)
        for i, s in enumerate(shapes):
            assert np.array_equal(got[i].export(), plain[i]), (chunk, s)
    ctx.tune("ip_chunk", 0)
    for i, (s, (A, B)) in enumerate(zip(shapes, mats)):
        assert np.array_equal(ctx.decrypt(ctx.import_ct(plain[i], 1, 2), *s), workloads.plain_matmul_mod(A, B, c.t))


def test_autotuner_keeps_bits_and_picks_a_setting():
    """The autotuner runs a small mixed batch under every setting of the
    transform radix and the launch-window size, finds the outputs
    bit-identical across settings (and equal to the oracle for one request),
    applies the fastest, and stores it for apply_cached."""
    import tempfile
    from paper_2405_02238_amd import autotune
    c = workloads.BATCHED
    shapes = [(8, 16, 24), (16, 8, 8), (24, 24, 16), (8, 40, 8), (32, 16, 40), (16, 16, 16)]
    ctx = hg.Context(c.N, c.t, c.L, c.alpha)
    ctx.keygen(c.seed, shapes)
    rng = np.random.default_rng(160)
    mats = [(rng.integers(-8, 9, size=(m, l)), rng.integers(-8, 9, size=(l, n))) for (m, l, n) in shapes]
    As = [ctx.encrypt(0, A, *s, nonce=i) for i, (s, (A, B)) in enumerate(zip(shapes, mats))]
    Bs = [ctx.encrypt(1, B, *s, nonce=i) for i, (s, (A, B)) in enumerate(zip(shapes, mats))]
    space = {"ntt_radix": [8, 16], "batch_window": [2, 0]}
    with tempfile.TemporaryDirectory() as d:
        cache = os.path.join(d, "tuned.json")
        rep = autotune.autotune(ctx, lambda: ctx.hegmm_batch(As, Bs, shapes), autotune.grid(space), reps=2,
                                cache=cache, tag="small")
        assert len(rep["all"]) == 4 and rep["best"]["knobs"] in autotune.grid(space)
        other = hg.Context(c.N, c.t, c.L, c.alpha)
        assert autotune.apply_cached(other, cache, "small") and not autotune.apply_cached(other, cache, "x")
    outs = ctx.hegmm_batch(As, Bs, shapes)
    P = Params(c.N, c.t, c.L, c.alpha)
    m, l, n = shapes[0]
    A, B = mats[0]
    ks = bgv.KeySet(P, c.seed, H.galois_elements(P, [shapes[0]]))
    pl = H.plan(m, l, n, P.S)
    want = flat(H.hegmm(ks, pl, H.encrypt_operand(ks, pl, 0, A, B, 0), H.encrypt_operand(ks, pl, 1, A, B, 0)))
    assert np.array_equal(outs[0].export(), want)
    for i, (s, (A, B)) in enumerate(zip(shapes, mats)):
        assert np.array_equal(ctx.decrypt(outs[i], *s), workloads.plain_matmul_mod(A, B, c.t)), s


def test_graph_replay_matches_eager(tiny):
    """A recorded batch (several launch windows) replays with the eager
    results, with other eager work and synchronisations between replays, and
    recomputes from operands refreshed in place."""
    ctx = tiny.ctx
    shapes = [(2, 5, 7), (5, 4, 2), (3, 11, 6), (4, 3, 5), (7, 7, 7)]
    rng = np.random.default_rng(77)
    mats = [(rng.integers(-8, 9, size=(m, l)), rng.integers(-8, 9, size=(l, n))) for (m, l, n) in shapes]
    As = [ctx.encrypt(0, A, *s, nonce=200 + i) for i, (s, (A, B)) in enumerate(zip(shapes, mats))]
    Bs = [ctx.encrypt(1, B, *s, nonce=200 + i) for i, (s, (A, B)) in enumerate(zip(shapes, mats))]
    eager = [o.export() for o in ctx.hegmm_batch(As, Bs, shapes)]
    ctx.tune("batch_window", 2)       # three launch windows, three private workspaces
    try:
        g = ctx.record_batch(As, Bs, shapes)
    finally:
        ctx.tune("batch_window", 64)
    zero = np.zeros_like(eager[0])
    for rep in range(3):
        for o in g.outputs:
            ctx.load_ct(o, zero)
        ctx.hegmm(As[rep], Bs[rep], *shapes[rep])     # eager work between replays
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        for i, s in enumerate(shapes):
            assert np.array_equal(g.outputs[i].export(), eager[i]), (rep, s)
    mats2 = [(rng.integers(-8, 9, size=(m, l)), rng.integers(-8, 9, size=(l, n))) for (m, l, n) in shapes]
    for i, (s, (A, B)) in enumerate(zip(shapes, mats2)):
        ctx.load_ct(As[i], ctx.encrypt(0, A, *s, nonce=300 + i).export())
        ctx.load_ct(Bs[i], ctx.encrypt(1, B, *s, nonce=300 + i).export())
    g.launch()
    torch.cuda.synchronize()
    again = [o.export() for o in ctx.hegmm_batch(As, Bs, shapes)]
    for i, (s, (A, B)) in enumerate(zip(shapes, mats2)):
        assert np.array_equal(g.outputs[i].export(), again[i]), s
        assert np.array_equal(ctx.decrypt(g.outputs[i], *s), workloads.plain_matmul_mod(A, B, tiny.P.t)), s
    g.close()


@pytest.mark.parametrize("method", [1, 3])
@pytest.mark.parametrize("shape", [(4, 3, 5), (3, 5, 2), (5, 3, 3), (2, 7, 6)])
def test_algorithm1_variant(shape, method):
    """Algorithm 1 (HEGMM, no duplication; column- or row-major whichever
    needs fewer key switches) against the oracle's Algorithm 1, bit for bit:
    sigma / tau applied by the client (method 1) or evaluated on the
    ciphertexts before the loop (method 3, Theorems 1 and 2)."""
    c = workloads.TINY
    m, l, n = shape
    ctx = hg.Context(c.N, c.t, c.L, c.alpha, method=method)
    ctx.keygen(c.seed, [shape])
    P = Params(c.N, c.t, c.L, c.alpha)
    ks = bgv.KeySet(P, c.seed, H.galois_elements(P, [shape], method=method))
    pl = H.plan(m, l, n, P.S, method=method)
    info = ctx.plan_info(m, l, n)
    assert info["transposed"] == int(pl.transposed) and info["K"] == l and info["d"] == 1
    assert info["rotations"] == len(pl.rotations(P.S))
    assert info["ks_terms"] == sum(1 for ts in pl.eps + pl.omega + [pl.sigma, pl.tau] for z, _ in ts if z % P.S)
    rng = np.random.default_rng(m + 10 * l + 100 * n)
    A = rng.integers(-8, 9, size=(m, l))
    B = rng.integers(-8, 9, size=(l, n))
    ca, cb = ctx.encrypt(0, A, m, l, n, nonce=4), ctx.encrypt(1, B, m, l, n, nonce=4)
    ox = H.encrypt_operand(ks, pl, 0, A, B, 4)
    oy = H.encrypt_operand(ks, pl, 1, A, B, 4)
    left, right = (cb, ca) if pl.transposed else (ca, cb)
    assert np.array_equal(left.export(), np.concatenate([flat(x) for x in ox]))
    assert np.array_equal(right.export(), np.concatenate([flat(y) for y in oy]))
    cc = ctx.hegmm(ca, cb, m, l, n)
    assert np.array_equal(cc.export(), flat(H.hegmm(ks, pl, ox, oy))), shape
    assert np.array_equal(ctx.decrypt(cc, m, l, n), workloads.plain_matmul_mod(A, B, c.t))


@pytest.mark.parametrize("method", [1, 3])
def test_algorithm1_eager_relin(method):
    """The variants compose: Algorithm 1 (client- or cloud-side sigma/tau)
    with every loop product relinearised on its own, against the oracle."""
    c = workloads.TINY
    m, l, n = 3, 4, 2
    ctx = hg.Context(c.N, c.t, c.L, c.alpha, method=method, relin=1)
    ctx.keygen(c.seed, [(m, l, n)])
    P = Params(c.N, c.t, c.L, c.alpha)
    ks = bgv.KeySet(P, c.seed, H.galois_elements(P, [(m, l, n)], method=method))
    pl = H.plan(m, l, n, P.S, method=method)
    rng = np.random.default_rng(17 + method)
    A = rng.integers(-8, 9, size=(m, l))
    B = rng.integers(-8, 9, size=(l, n))
    ca, cb = ctx.encrypt(0, A, m, l, n, nonce=6), ctx.encrypt(1, B, m, l, n, nonce=6)
    ox = H.encrypt_operand(ks, pl, 0, A, B, 6)
    oy = H.encrypt_operand(ks, pl, 1, A, B, 6)
    cc = ctx.hegmm(ca, cb, m, l, n)
    assert np.array_equal(cc.export(), flat(H.hegmm(ks, pl, ox, oy, eager=True)))
    assert np.array_equal(ctx.decrypt(cc, m, l, n), workloads.plain_matmul_mod(A, B, c.t))


def test_execution_knobs_bit_identical():
    """Every execution knob changes only the schedule: pipelined passes on a
    second stream, split-row transforms, fused or unfused chains, launch
    windows, the XCD row map -- the 64x32x48 product and a small batch keep
    their bits."""
    c = workloads.HEADLINE
    m, l, n = 64, 32, 48
    A, B = workloads.headline_operands()
    ctx = hg.Context(c.N, c.t, c.L, c.alpha)
    shapes = [(m, l, n), (8, 24, 16), (40, 8, 8)]
    ctx.keygen(c.seed, shapes)
    ca, cb = ctx.encrypt(0, A, m, l, n, nonce=1), ctx.encrypt(1, B, m, l, n, nonce=1)
    rng = np.random.default_rng(5)
    mats = [(rng.integers(-8, 9, size=(a, b)), rng.integers(-8, 9, size=(b, d))) for (a, b, d) in shapes[1:]]
    As = [ca] + [ctx.encrypt(0, X, *s, nonce=2 + i) for i, (s, (X, Y)) in enumerate(zip(shapes[1:], mats))]
    Bs = [cb] + [ctx.encrypt(1, Y, *s, nonce=2 + i) for i, (s, (X, Y)) in enumerate(zip(shapes[1:], mats))]
    ref_one = ctx.hegmm(ca, cb, m, l, n).export()
    ref_batch = [o.export() for o in ctx.hegmm_batch(As, Bs, shapes)]
    settings = [{"pipeline": 2}, {"pipeline": 3, "fuse_rows": 0}, {"split_rows": 64, "fuse_rows": 0},
                {"fuse_rows": 4096}, {"batch_window": 1}, {"ip_chunk": 16}, {"ip_chunk": 4, "batch_window": 0},
                {"ip_order": 0}, {"ntt_radix": 16}, {"ntt_radix": 16, "fuse_rows": 0, "pipeline": 2},
                {"half_rows": 0}, {"half_rows": 4096, "fuse_rows": 4096}, {"half_rows": 0, "ntt_radix": 16},
                {"xcd_rows": 0}, {"xcd_rows": 0, "ntt_radix": 16, "fuse_rows": 0}]
    defaults = {"pipeline": 1, "fuse_rows": 256, "split_rows": 0, "batch_window": 64, "ip_chunk": 0, "ip_order": 1,
                "ntt_radix": 0, "half_rows": 128, "xcd_rows": 1}
    with pytest.raises(hg.HGError):
        ctx.tune("xcd_rows", 2)
    for st in settings:
        for k, v in st.items():
            ctx.tune(k, v)
        assert np.array_equal(ctx.hegmm(ca, cb, m, l, n).export(), ref_one), st
        got = ctx.hegmm_batch(As, Bs, shapes)
        for i, s in enumerate(shapes):
            assert np.array_equal(got[i].export(), ref_batch[i]), (st, s)
        for k in st:
            ctx.tune(k, defaults[k])


def test_launch_timing_counts_and_bits(tiny):
    """Launch timing (hg_set_timing mode 2) keeps one event pair per
    transform-pass inner-product launch across calls, changes no bits, leaves
    graph recording untimed, and starts a new tally once read."""
    m, l, n = 4, 3, 5
    A, B = workloads.tiny_operands()
    ctx = tiny.ctx
    ca, cb = ctx.encrypt(0, A, m, l, n, nonce=1), ctx.encrypt(1, B, m, l, n, nonce=1)
    ref = ctx.hegmm(ca, cb, m, l, n).export()
    ctx.set_timing(True)
    ctx.hegmm(ca, cb, m, l, n)
    per_call = int(ctx.last_timing()["ip_launches"])
    ctx.set_timing(False)
    assert per_call >= 1
    ctx.set_launch_timing(True)
    try:
        outs = [ctx.hegmm(ca, cb, m, l, n) for _ in range(3)]
        g = ctx.record_batch([ca], [cb], [(m, l, n)])
        g.launch()
        torch.cuda.synchronize()
        lt = ctx.launch_timing()
        again = ctx.launch_timing()
    finally:
        ctx.set_launch_timing(False)
    # three eager calls; the graph's first (eager) pass is not timed either
    assert lt["ip_launches"] == 3 * per_call
    assert lt["ip_kernel"] > 0
    assert again == {"ip_kernel": 0.0, "ip_launches": 0, "md_fwd_kernel": 0.0, "md_fwd_launches": 0}
    # few rows: the division by P runs fused, so no forward transform is timed
    assert lt["md_fwd_launches"] == 0
    for o in outs + list(g.outputs):
        assert np.array_equal(o.export(), ref)
    g.close()
