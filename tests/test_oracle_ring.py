"""Pins for the oracle's ring layer: each check compares against a definition
written out independently here (direct evaluation, schoolbook products,
published test vectors, brute-force searches), never against the oracle's
own formulas."""
import math
import random

import numpy as np
import pytest

from oracle import ring
from oracle.ring import Params

Q50 = 1125899906826241          # a 50-bit prime = 1 mod 2^11 (first special prime at N <= 1024)


def direct_eval(a, psi, q):
    """a(psi^(2i+1)) for every i, by Horner's rule on each point."""
    N = len(a)
    out = []
    for i in range(N):
        x = pow(psi, 2 * i + 1, q)
        acc = 0
        for c in reversed(a):
            acc = (acc * x + int(c)) % q
        out.append(acc)
    return out


def negacyclic_product(a, b, q):
    """Plain polynomial product, then X^N = -1."""
    N = len(a)
    full = [0] * (2 * N)
    for i in range(N):
        for j in range(N):
            full[i + j] += int(a[i]) * int(b[j])
    return [(full[k] - full[k + N]) % q for k in range(N)]


@pytest.mark.parametrize("N", [8, 16, 32, 64])
def test_ntt_is_evaluation_at_odd_powers(N):
    psi = ring.primitive_2n_root(Q50, N)
    assert pow(psi, N, Q50) == Q50 - 1
    rng = random.Random(N)
    a = [rng.randrange(Q50) for _ in range(N)]
    got = ring.ntt(np.array([a], dtype=np.uint64), np.array([Q50], dtype=np.uint64),
                   np.array([psi], dtype=np.uint64))[0]
    assert [int(x) for x in got] == direct_eval(a, psi, Q50)


@pytest.mark.parametrize("N", [8, 16, 64])
def test_transform_product_matches_schoolbook(N):
    P = Params(N, 12289, 2, 1)
    rng = random.Random(100 + N)
    a = np.array([[rng.randrange(q) for _ in range(N)] for q in P.q], dtype=np.uint64)
    b = np.array([[rng.randrange(q) for _ in range(N)] for q in P.q], dtype=np.uint64)
    got = ring.polymul(P, a, b)
    for r, q in enumerate(P.q):
        assert [int(x) for x in got[r]] == negacyclic_product(a[r], b[r], q)
        assert [int(x) for x in ring.schoolbook(a[r], b[r], q)] == negacyclic_product(a[r], b[r], q)


def test_inverse_transform_roundtrip():
    P = Params(256, 12289, 3, 1)
    rng = np.random.default_rng(1)
    a = np.stack([rng.integers(0, q, P.N, dtype=np.uint64) for q in P.ext])
    back = ring.intt(ring.ntt(a, P.ext_arr, P.psi_ext), P.ext_arr, P.psi_ext)
    assert (back == a).all()


def test_automorphism_is_substitution():
    """or_automorph: a(X) -> a(X^g) computed by substituting and reducing X^N = -1."""
    N, q, g = 16, Q50, 5 ** 3 % 32
    rng = random.Random(7)
    a = [rng.randrange(q) for _ in range(N)]
    expect = [0] * N
    for j, c in enumerate(a):
        e = j * g
        sign = -1 if (e // N) % 2 else 1
        expect[e % N] = (expect[e % N] + sign * c) % q
    got = ring.automorph(np.array([a], dtype=np.uint64), g, np.array([q], dtype=np.uint64))[0]
    assert [int(x) for x in got] == expect


@pytest.mark.parametrize("bits", [50, 40])
def test_primes_rule(bits):
    for N, L, alpha in [(1024, 3, 1), (8192, 4, 1), (16384, 6, 2), (32768, 8, 2)]:
        ps = ring.ntt_primes(N, L + alpha, bits)
        assert ps == sorted(ps, reverse=True)
        for p in ps:
            assert 2 ** (bits - 1) < p < 2 ** bits and p % (2 * N) == 1
            # an independent probable-prime check (Fermat, bases other than MR's)
            assert all(pow(b, p - 1, p) == 1 for b in (41, 43, 47, 53))
        # no skipped candidate above the first or between consecutive primes
        for hi, lo in zip([2 ** bits] + ps, ps):
            for c in range(lo + 2 * N, hi, 2 * N):
                assert not all(pow(b, c - 1, c) == 1 for b in (2, 3, 5, 7))


def test_zeta_is_smallest_root():
    for N, t in [(1024, 12289), (8192, 65537), (16384, 65537), (32768, 786433)]:
        z = ring.smallest_2n_root(t, N)
        assert pow(z, N, t) == t - 1
        assert all(pow(x, N, t) != t - 1 for x in range(2, z))


def test_splitmix64_published_vectors():
    # SplitMix64 seeded with 0: the first three outputs of the reference generator
    s0 = 0
    outs = [ring.mix64((s0 + k * 0x9E3779B97F4A7C15) % 2 ** 64) for k in (1, 2, 3)]
    assert outs == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_gaussian_table_and_samples():
    cdt = ring.gaussian_cdt()
    assert len(cdt) == 38 and all(x < y for x, y in zip(cdt, cdt[1:]))
    # symmetric: F(-1) + F(0) = 1 (in units of 2^-64, up to the two floors)
    assert abs(cdt[18] + cdt[19] - 2 ** 64) <= 2
    rho = [math.exp(-x * x / (2 * 3.2 ** 2)) for x in range(-19, 20)]
    z = sum(rho)
    assert abs(cdt[19] / 2 ** 64 - sum(rho[:20]) / z) < 1e-12
    P = Params(1024, 12289, 1, 1)
    xs = np.concatenate([ring.sample_gauss(P, ring.stream_seed(9, 9, i), 0) for i in range(64)])
    assert xs.min() >= -19 and xs.max() <= 19
    assert abs(xs.mean()) < 0.05
    assert abs(xs.std() - 3.2) < 0.05


def test_ternary_and_uniform_samples():
    t = ring.sample_ternary(ring.stream_seed(1, 2, 3), 0, 30000)
    counts = [int((t == v).sum()) for v in (-1, 0, 1)]
    assert all(abs(c - 10000) < 400 for c in counts)
    q = np.array([Q50], dtype=np.uint64)
    u = ring.sample_uniform(ring.stream_seed(4, 5, 6), 0, q, 30000)[0]
    assert int(u.max()) < Q50
    assert abs(float(u.mean()) / Q50 - 0.5) < 0.01


@pytest.mark.parametrize("N,t", [(16, 97), (64, 12289), (1024, 12289)])
def test_encode_matches_direct_evaluation(N, t):
    P = Params(N, t, 1, 1)
    rng = random.Random(N)
    slots = [rng.randrange(t) for _ in range(P.S)]
    mu = [int(x) for x in ring.encode(P, slots)]
    assert len(mu) == N and all(0 <= c < t for c in mu)
    check = range(P.S) if N <= 64 else range(0, P.S, 37)
    for s in check:
        for e, want in ((pow(5, s, 2 * N), slots[s]), ((-pow(5, s, 2 * N)) % (2 * N), 0)):
            x = pow(P.zeta, e, t)
            val = 0
            for c in reversed(mu):
                val = (val * x + c) % t
            assert val == want
    assert ring.decode(P, np.array(mu)) == slots


@pytest.mark.parametrize("z", [1, 3, -1, -5, 17])
def test_plaintext_rotation_is_galois_5_power(z):
    """decode(mu(X^(5^z))) is the slot vector rotated left by z: exact, no noise."""
    P = Params(64, 12289, 1, 1)
    rng = random.Random(z + 50)
    slots = [rng.randrange(P.t) for _ in range(P.S)]
    mu = ring.encode(P, slots)
    g = P.galois(z)
    rot = ring.automorph(np.array([mu], dtype=np.uint64), g, np.array([P.t], dtype=np.uint64))[0]
    assert ring.decode(P, rot) == [slots[(s + z) % P.S] for s in range(P.S)]


def test_centered_lift():
    assert list(ring.lift_centered(np.array([0, 1, 6144, 6145, 12288]), 12289)) == [0, 1, 6144, -6144, -1]
