"""Pins for the oracle's BGV layer.

Key switching, rotation and relinearisation have no printed values in the
paper; they are pinned by what the mathematics fixes: decryptions of every
primitive (slot-wise sums, products, rotations), exactness of the division by
P (checked with big integers), the key relation u0 + u1 s = P c s' + t e, and
bit-identities that must hold by construction."""
import math
import random

import numpy as np
import pytest

from oracle import bgv, ring
from oracle.ring import Params


def crt(rows, primes):
    """Big-integer CRT of residue rows, centered in (-M/2, M/2)."""
    M = 1
    for p in primes:
        M *= p
    out = []
    for k in range(len(rows[0])):
        x = 0
        for r, p in zip(rows, primes):
            hat = M // p
            x += int(r[k]) * hat * pow(hat % p, -1, p)
        x %= M
        out.append(x - M if x > M // 2 else x)
    return out


@pytest.fixture(scope="module", params=[(64, 12289, 3, 1), (64, 12289, 4, 2), (128, 12289, 3, 2)],
                ids=["a1", "a2", "a2-ragged"])
def setup(request):
    N, t, L, alpha = request.param
    P = Params(N, t, L, alpha)
    zs = [1, 2, 5, -1, -3, P.S - 1, 7]
    ks = bgv.KeySet(P, 424242, [P.galois(z) for z in zs])
    return P, ks


def rand_slots(P, seed):
    rng = random.Random(seed)
    return [rng.randrange(P.t) for _ in range(P.S)]


def test_roundtrip(setup):
    P, ks = setup
    v = rand_slots(P, 1)
    ct = bgv.encrypt_slots(ks, v, nonce=5)
    assert bgv.decrypt_slots(ks, ct) == v
    assert all(int(c.max()) < q for c, q in zip(ct[0], P.q))


def test_encrypt_is_rlwe_sample(setup):
    """c0 + c1 s - lift(mu) is t times a small error (|e| <= 19)."""
    P, ks = setup
    v = rand_slots(P, 2)
    mu = ring.encode(P, v)
    ct = bgv.encrypt_slots(ks, v, nonce=6)
    acc = ring.add(ct[0], ring.polymul(P, ct[1], ks.sk.s_ext[:P.L]), P.q_arr)
    vals = crt(acc, P.q)
    lifted = ring.lift_centered(mu, P.t)
    for x, m in zip(vals, lifted):
        d = x - int(m)
        assert d % P.t == 0 and abs(d // P.t) <= 19


def test_add_and_cmult(setup):
    P, ks = setup
    a, b = rand_slots(P, 3), rand_slots(P, 4)
    ca, cb = bgv.encrypt_slots(ks, a, nonce=1), bgv.encrypt_slots(ks, b, nonce=2)
    assert bgv.decrypt_slots(ks, bgv.he_add(P, ca, cb)) == [(x + y) % P.t for x, y in zip(a, b)]
    mask = [1 if (s * 7) % 3 == 0 else 0 for s in range(P.S)]
    got = bgv.decrypt_slots(ks, bgv.he_cmult(P, ca, bgv.Mask(P, mask)))
    assert got == [x * m for x, m in zip(a, mask)]


@pytest.mark.parametrize("z", [1, 2, 5, -1, -3, 7])
def test_rotation_decrypts_to_left_rotation(setup, z):
    P, ks = setup
    v = rand_slots(P, 10 + z)
    ct = bgv.encrypt_slots(ks, v, nonce=3)
    assert bgv.decrypt_slots(ks, bgv.rotate(P, ks, ct, z)) == [v[(s + z) % P.S] for s in range(P.S)]


def test_rotation_identities(setup):
    P, ks = setup
    v = rand_slots(P, 20)
    ct = bgv.encrypt_slots(ks, v, nonce=4)
    # rotation by 0 is the identity, bit for bit, with no key switch
    r0 = bgv.rotate(P, ks, ct, 0)
    assert all((x == y).all() for x, y in zip(r0, ct))
    # z and z + S name the same Galois element: identical bits
    a = bgv.rotate(P, ks, ct, 2)
    b = bgv.rotate(P, ks, ct, 2 + P.S)
    assert all((x == y).all() for x, y in zip(a, b))
    # composition: Rot(Rot(ct, 1), 1) decrypts like Rot(ct, 2)
    c = bgv.rotate(P, ks, bgv.rotate(P, ks, ct, 1), 1)
    assert bgv.decrypt_slots(ks, c) == bgv.decrypt_slots(ks, a)
    # Rot(., -1) undoes Rot(., 1)
    d = bgv.rotate(P, ks, bgv.rotate(P, ks, ct, 1), -1)
    assert bgv.decrypt_slots(ks, d) == v


def test_mult_and_relin(setup):
    P, ks = setup
    a, b = rand_slots(P, 30), rand_slots(P, 31)
    ca, cb = bgv.encrypt_slots(ks, a, nonce=7), bgv.encrypt_slots(ks, b, nonce=8)
    t3 = bgv.tensor(P, ca, cb)
    want = [(x * y) % P.t for x, y in zip(a, b)]
    assert ring.decode(P, bgv.decrypt_poly(ks, t3)) == want
    assert bgv.decrypt_slots(ks, bgv.relinearize(P, ks, t3)) == want


def test_masked_rot_sum(setup):
    P, ks = setup
    v = rand_slots(P, 40)
    ct = bgv.encrypt_slots(ks, v, nonce=9)
    m1 = [1 if s < P.S // 3 else 0 for s in range(P.S)]
    m2 = [1 - x for x in m1]
    out = bgv.rot_sum(P, ks, ct, [(5, bgv.Mask(P, m1)), (-3, bgv.Mask(P, m2)), (0, bgv.Mask(P, m2))])
    want = [(m1[s] * v[(s + 5) % P.S] + m2[s] * v[(s - 3) % P.S] + m2[s] * v[s]) % P.t for s in range(P.S)]
    assert bgv.decrypt_slots(ks, out) == want


def test_rotate_is_the_one_term_rot_sum(setup):
    """HE-Rot written out on its own (one division by P) and the deferred
    rotation sum with a single unmasked term are the same computation: equal
    bits, for rotated and unrotated terms."""
    P, ks = setup
    ct = bgv.encrypt_slots(ks, rand_slots(P, 41), nonce=12)
    for z in (1, -3, 7, 0, P.S):
        a = bgv.rotate(P, ks, ct, z)
        b = bgv.rot_sum(P, ks, ct, [(z, None)])
        assert all((x == y).all() for x, y in zip(a, b)), z


def test_paper_order_lin_transform(setup):
    """Eq. (lintrans) in the paper's primitive order (HE-Rot, HE-CMult, HE-Add
    per diagonal) decrypts to the masked slot sum; the deferred division by P
    gives the same plaintext with different bits.  The noise of the two orders
    agrees within a quarter bit: in both it is dominated by the mask times the
    input's own noise, and they differ only in where one rounding term of the
    division by P enters."""
    P, ks = setup
    v = rand_slots(P, 42)
    ct = bgv.encrypt_slots(ks, v, nonce=13)
    m1 = [1 if s < P.S // 3 else 0 for s in range(P.S)]
    m2 = [1 - x for x in m1]
    terms = [(5, bgv.Mask(P, m1)), (-3, bgv.Mask(P, m2)), (0, bgv.Mask(P, m2))]
    paper = bgv.lin_transform(P, ks, ct, terms)
    deferred = bgv.rot_sum(P, ks, ct, terms)
    want = [(m1[s] * v[(s + 5) % P.S] + m2[s] * v[(s - 3) % P.S] + m2[s] * v[s]) % P.t for s in range(P.S)]
    assert bgv.decrypt_slots(ks, paper) == want
    assert bgv.decrypt_slots(ks, deferred) == want
    assert any((x != y).any() for x, y in zip(paper, deferred))
    mu = ring.encode(P, want)
    assert abs(bgv.noise_bits(ks, deferred, mu) - bgv.noise_bits(ks, paper, mu)) <= 0.25
    # a transform of one unmasked diagonal is the rotation itself in both orders
    one = bgv.lin_transform(P, ks, ct, [(7, None)])
    assert all((x == y).all() for x, y in zip(one, bgv.rotate(P, ks, ct, 7)))


def test_moddown_is_exact_division(setup):
    """out * P = u - delta with delta = 0 (mod t) and |delta| <= t * alpha * P / 2."""
    P, ks = setup
    rng = np.random.default_rng(5)
    u = np.stack([rng.integers(0, p, P.N, dtype=np.uint64) for p in P.ext])
    out = ring.moddown(P, u)
    QP = P.Q * P.P
    u_int = crt(u, P.ext)
    o_int = crt(out, P.q)
    for ui, oi in zip(u_int, o_int):
        delta = (ui - oi * P.P) % QP
        if delta > QP // 2:
            delta -= QP
        assert delta % P.t == 0
        assert abs(delta) <= P.t * P.alpha * P.P // 2


def test_modup_lifts_the_digit(setup):
    """y_j = c mod each digit prime, and y_j is a small multiple-of-digit lift."""
    P, ks = setup
    rng = np.random.default_rng(6)
    c = np.stack([rng.integers(0, q, P.N, dtype=np.uint64) for q in P.q])
    for j, (d0, d1) in enumerate(P.digits):
        y = ring.modup_digit(P, c, j)
        D = 1
        for r in range(d0, d1):
            D *= P.q[r]
            assert (y[r] == c[r]).all()
        vals = crt(y, P.ext)
        digit_vals = crt(c[d0:d1], P.q[d0:d1])
        for v, dv in zip(vals, digit_vals):
            assert (v - dv) % D == 0
            assert abs(v) <= (d1 - d0) * D // 2


def test_switch_key_relation(setup):
    """The inner product with a rotation key satisfies u0 + u1 s = P c s' + t e (mod QP)."""
    P, ks = setup
    g = P.galois(1)
    rng = np.random.default_rng(7)
    c = np.stack([rng.integers(0, q, P.N, dtype=np.uint64) for q in P.q])
    u0, u1 = bgv.ks_inner(P, c, ks.rot[g])
    u0c = ring.intt(u0, P.ext_arr, P.psi_ext)
    u1c = ring.intt(u1, P.ext_arr, P.psi_ext)
    lhs = ring.add(u0c, ring.polymul(P, u1c, ks.sk.s_ext), P.ext_arr)
    sg = ring.automorph(ks.sk.s_ext, g, P.ext_arr)
    c_int = crt(c, P.q)
    c_ext = np.array([[x % p for x in c_int] for p in P.ext], dtype=np.uint64)
    rhs = ring.scale(ring.polymul(P, c_ext, sg), [P.P] * (P.L + P.alpha), P.ext_arr)
    diff = crt(ring.sub(lhs, rhs, P.ext_arr), P.ext)
    maxD = max(math.prod(P.q[d0:d1]) for d0, d1 in P.digits)
    bound = P.t * 19 * P.N * P.beta * P.alpha * maxD
    for x in diff:
        assert x % P.t == 0
        assert abs(x) < bound


def test_hoisting_is_bit_neutral(setup):
    """ModUp commutes with the automorphism exactly (centered lifts are odd
    functions for odd moduli), so a GPU may lift once and permute after."""
    P, ks = setup
    rng = np.random.default_rng(8)
    c = np.stack([rng.integers(0, q, P.N, dtype=np.uint64) for q in P.q])
    for z in (1, -3, 7):
        g = P.galois(z)
        for j in range(P.beta):
            a = ring.modup_digit(P, ring.automorph(c, g, P.q_arr), j)
            b = ring.automorph(ring.modup_digit(P, c, j), g, P.ext_arr)
            assert (a == b).all()


def test_noise_stays_in_budget(setup):
    P, ks = setup
    v = rand_slots(P, 50)
    ct = bgv.encrypt_slots(ks, v, nonce=11)
    r = bgv.rotate(P, ks, ct, 5)
    mu = ring.encode(P, [v[(s + 5) % P.S] for s in range(P.S)])
    assert bgv.noise_bits(ks, r, mu) < math.log2(P.Q) - 2


# ---------------------------------------------------------------------------
# modulus switching
# ---------------------------------------------------------------------------

def _switch_bound(P, ks, nb_in, lv):
    """The rescaling bound of BGV modulus switching from level lv to lv - 1:
    |v'| <= k (|v|) / q + t (1 + |s|_1) / 2, v the centered decryption before
    reduction mod t (|v| <= 2^nb_in + t / 2), plus t / 2 for the message."""
    q = P.q[lv - 1]
    k = q % P.t
    s1 = int(np.abs(np.asarray(ks.sk.s, dtype=np.int64)).sum())
    return k * (2.0 ** nb_in + P.t / 2) / q + P.t * (1 + s1) / 2 + P.t / 2


def test_mod_switch_keeps_plaintext_and_bounds_noise():
    """Dropping one and two primes keeps the decrypted slots, leaves L - drop
    rows, and the noise obeys the closed-form rescaling bound at each step."""
    P = Params(1024, 12289, 3, 1)
    ks = bgv.KeySet(P, 5, [])
    rng = np.random.default_rng(11)
    for nonce in range(3):
        v = [int(x) for x in rng.integers(0, P.t, P.S)]
        c = bgv.encrypt_slots(ks, v, nonce=nonce)
        mu = bgv.decrypt_poly(ks, c)
        nb = bgv.noise_bits(ks, c, mu)
        cur = c
        for lv in (P.L, P.L - 1):
            nxt = bgv.mod_switch(P, cur, 1)
            assert all(x.shape == (lv - 1, P.N) for x in nxt)
            assert bgv.decrypt_slots(ks, nxt) == v
            nb2 = bgv.noise_bits(ks, nxt, mu)
            assert 2.0 ** nb2 <= _switch_bound(P, ks, nb, lv)
            cur, nb = nxt, nb2
        two = bgv.mod_switch(P, c, 2)
        assert all(np.array_equal(a, b) for a, b in zip(two, cur))


def test_mod_switch_of_a_product():
    """A relinearised product (large noise) switched down one prime: the
    plaintext is kept and the noise shrinks by about q / k."""
    P = Params(1024, 12289, 3, 1)
    ks = bgv.KeySet(P, 6, [])
    rng = np.random.default_rng(12)
    a = [int(x) for x in rng.integers(0, P.t, P.S)]
    b = [int(x) for x in rng.integers(0, P.t, P.S)]
    ca, cb = bgv.encrypt_slots(ks, a, nonce=1), bgv.encrypt_slots(ks, b, nonce=2)
    prod = bgv.he_mult(P, ks, ca, cb)
    want = [(x * y) % P.t for x, y in zip(a, b)]
    assert bgv.decrypt_slots(ks, prod) == want
    mu = bgv.decrypt_poly(ks, prod)
    nb = bgv.noise_bits(ks, prod, mu)
    sw = bgv.mod_switch(P, prod, 1)
    assert bgv.decrypt_slots(ks, sw) == want
    nb2 = bgv.noise_bits(ks, sw, mu)
    assert 2.0 ** nb2 <= _switch_bound(P, ks, nb, P.L)
    assert nb2 < nb
    with pytest.raises(ValueError):
        bgv.mod_switch(P, prod, P.L)
