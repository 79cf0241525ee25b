"""The FP64 modular arithmetic of the transform kernels, emulated operation by
operation on the CPU, stays exact under the kernels' lazy reduction schedule.

The kernels keep residues in doubles and rely on three facts: a product of
two doubles is split exactly into h + l with one fused multiply-add; the
quotient estimate rint(h * fl(1/q)) is within one of the true quotient; and
every value that must be exact (sums, the fused remainder h - e q, r + l) is
an integer below 2^53.  The forward transforms reduce on every fourth stage
(3, 7, 11, ... and the last), the inverse transforms reduce their sums on
every second stage (odd stages and the last).  This test runs both butterfly
networks, with IEEE doubles for every rounded operation (Python floats) and
exact integers for every fused one, on random and on extreme inputs and
twiddles, asserts that no step that must be exact rounds, and compares the
results with the same networks in exact modular arithmetic.  It restates the
arithmetic only; the library's kernels are checked bit for bit against the
oracle by the GPU tests.
"""
import random

import pytest

Q = 1125899906826241          # a prime just below 2^50, 1 (mod 2^14)
QI = 1.0 / Q
LIM = 1 << 53


def _fma_exact(a: float, b: float, c: float) -> float:
    """fma(a, b, c) of integer-valued doubles, asserting the result needs no rounding."""
    v = int(a) * int(b) + int(c)
    assert abs(v) < LIM, v
    return float(v)


def _add(a: float, b: float) -> float:
    v = int(a) + int(b)
    assert abs(v) < LIM, v
    return float(v)


def _rint(x: float) -> float:
    return float(round(x))    # round half to even, as rint in the default mode


def mulm(a: float, b: float, q: int = Q) -> float:
    h = a * b                                   # rounded product
    l = float(int(a) * int(b) - int(h))         # its exact error (fma(a, b, -h))
    assert abs(l) < LIM
    e = _rint(h * (1.0 / q))
    r = _fma_exact(-e, q, h)
    return _add(r, l)


def redm(x: float, q: int = Q) -> float:
    assert abs(x) < LIM
    return _fma_exact(-_rint(x * (1.0 / q)), q, x)


def forward(x, tw, exact):
    """Cooley-Tukey stages, natural-order input; stage g pairs i and i + N/2^(g+1)
    with twiddle tw[2^g + block]."""
    n = len(x)
    logn = n.bit_length() - 1
    worst = 0
    for g in range(logn):
        half = n >> (g + 1)
        red = g % 4 == 3 or g == logn - 1
        for blk in range(1 << g):
            w = tw[(1 << g) + blk]
            base = blk * 2 * half
            for i in range(base, base + half):
                if exact:
                    t = x[i + half] * w % Q
                    x[i], x[i + half] = (x[i] + t) % Q, (x[i] - t) % Q
                    continue
                t = mulm(x[i + half], w)
                a, b = _add(x[i], t), _add(x[i], -t)
                worst = max(worst, abs(a), abs(b))
                x[i], x[i + half] = (redm(a), redm(b)) if red else (a, b)
    return worst


def inverse(x, tw, exact, every_stage=False):
    """Gentleman-Sande stages, stage g pairs i and i + 2^g with twiddle
    tw[n / 2^(g+1) + block].  The one-workgroup rows reduce their sums on odd
    stages and the last; the two-pass rows (every_stage) on every stage."""
    n = len(x)
    logn = n.bit_length() - 1
    worst = 0
    for g in range(logn):
        d = 1 << g
        red = (g & 1) or g == logn - 1 or every_stage
        for blk in range(n >> (g + 1)):
            w = tw[(n >> (g + 1)) + blk]
            base = blk * 2 * d
            for i in range(base, base + d):
                X, Y = x[i], x[i + d]
                if exact:
                    x[i], x[i + d] = (X + Y) % Q, (X - Y) * w % Q
                    continue
                s, df = _add(X, Y), _add(X, -Y)
                worst = max(worst, abs(s), abs(df))
                x[i] = redm(s) if red else s
                x[i + d] = mulm(df, w)
    return worst


def _case(n, kind, seed):
    rng = random.Random(seed)
    half = (Q - 1) // 2
    if kind == "random":
        x = [float(rng.randrange(-(Q - 1), Q)) for _ in range(n)]
        tw = [float(rng.randrange(-half, half + 1)) for _ in range(n)]
    else:   # extreme: inputs at +-(q - 1), twiddles at +-(q - 1)/2
        x = [float((Q - 1) * (1 if (i * 7 + seed) % 3 else -1)) for i in range(n)]
        tw = [float(half * (1 if (i + seed) % 2 else -1)) for i in range(n)]
    return x, tw


@pytest.mark.parametrize("n", [8192, 16384])
@pytest.mark.parametrize("kind", ["random", "extreme"])
def test_lazy_schedule_exact(n, kind):
    for direction in (forward, inverse):
        x, tw = _case(n, kind, n + len(kind))
        ref = [int(v) % Q for v in x]
        twi = [int(w) % Q for w in tw]
        direction(ref, twi, exact=True)
        worst = direction(x, tw, exact=False)
        assert worst < LIM
        assert all((int(a) - b) % Q == 0 for a, b in zip(x, ref)), direction.__name__
        # the outputs: reduced sums and twiddle products, below 2q
        assert max(abs(v) for v in x) < 2 * Q, direction.__name__


def test_two_pass_schedule_exact():
    """The 32768-point rows run in two passes (a column pass of stages 0..7,
    reducing at stages 3 and 7, then a block pass of stages 8..14, reducing at
    11 and the last): the same every-fourth-stage rule as the one-workgroup
    rows.  Their inverse reduces the sums on every stage.  (The emulation runs
    the stages in order; the passes only regroup the butterflies of a stage.)"""
    n = 32768
    for kind in ("random", "extreme"):
        x, tw = _case(n, kind, 7 + len(kind))
        ref = [int(v) % Q for v in x]
        twi = [int(w) % Q for w in tw]
        forward(ref, twi, exact=True)
        assert forward(x, tw, exact=False) < LIM
        assert all((int(a) - b) % Q == 0 for a, b in zip(x, ref))
        x, tw = _case(n, kind, 9 + len(kind))
        ref = [int(v) % Q for v in x]
        inverse(ref, [int(w) % Q for w in tw], exact=True)
        assert inverse(x, tw, exact=False, every_stage=True) < LIM
        assert all((int(a) - b) % Q == 0 for a, b in zip(x, ref))


# The first twelve primes below 2^50 that are 1 (mod 2^16): the primes of
# rings up to N = 32768, the largest the library builds.
BIG = [1125899904679937, 1125899903827969, 1125899903500289, 1125899903107073,
       1125899902124033, 1125899901665281, 1125899899174913, 1125899896160257,
       1125899887312897, 1125899886395393, 1125899885740033, 1125899885412353]


def _worst_product(q: int, rng: random.Random) -> tuple:
    """Operands below q whose FP64 modular product has the largest |result|
    of a few thousand tries near the rounding boundary of the quotient."""
    best = (0.0, 1.0, 1.0)
    for _ in range(3000):
        a = float(rng.randrange(q // 2, q) * rng.choice((1, -1)))
        b = float(rng.randrange(q // 2, q))
        r = mulm(a, b, q)
        if abs(r) > abs(best[0]):
            best = (r, a, b)
    return best


@pytest.mark.parametrize("beta", [4, 8, 9, 12])
def test_inner_product_digit_sums_exact(beta):
    """The key-switch inner products add BETA digit products before one
    reduction, and with BETA above 9 reduce after every 8th product: with
    products all of one sign and near their largest size, no partial sum
    reaches 2^53 and the result is the exact modular sum.  The proven bound
    |mulm| < 0.875 q caps a run of 8 products plus a reduced value at 7.5 q
    and a run of 9 at 7.9 q, both below 8 q <= 2^53."""
    q = BIG[0]
    rng = random.Random(beta)
    r, a, b = _worst_product(q, rng)
    assert abs(r) > 0.45 * q
    ys = [a] * beta
    ks = [b] * beta
    acc = 0.0
    worst = 0.0
    for j in range(beta):
        acc = _add(acc, mulm(ys[j], ks[j], q))
        worst = max(worst, abs(acc))
        if beta > 9 and j % 8 == 7 and j + 1 < beta:
            acc = redm(acc, q)
    acc = redm(acc, q)
    assert worst < LIM
    assert (int(acc) - beta * int(a) * int(b)) % q == 0
    assert 8 * 0.875 * q + (q / 2 + 1) < LIM and 9 * 0.875 * q < LIM
    if beta > 9:
        assert beta * 0.875 * q > LIM     # an unreduced sum would not be provably exact


@pytest.mark.parametrize("alpha", [2, 3, 4])
def test_two_prime_digit_lift_and_delta_sums_exact(alpha):
    """The digit lift of a digit of alpha primes (LOAD_MODUP) adds alpha
    products of a centered residue (below q_s / 2) and an uncentered
    constant (D_j / q_s mod q_r) before one reduction; the correction of the
    division by P (LOAD_DELTA) adds alpha products of a centered r_k and
    t (P / p_k) mod q_i.  With extreme operands every partial sum stays
    below 2^53 and the reduced results are the exact modular sums."""
    rng = random.Random(alpha)
    digit = BIG[:alpha]
    r_prime = BIG[alpha]
    for trial in range(200):
        acc = 0.0
        exact = 0
        for s in digit:
            ct = float(rng.choice(((s - 1) // 2, -((s - 1) // 2), rng.randrange(-(s // 2), s // 2))))
            hat = float(rng.choice((r_prime - 1, rng.randrange(r_prime))))
            acc = _add(acc, mulm(ct, hat, r_prime))
            exact += int(ct) * int(hat)
        assert abs(acc) < LIM
        assert (int(redm(acc, r_prime)) - exact) % r_prime == 0
    for trial in range(200):
        qi = BIG[-1]
        acc = 0.0
        exact = 0
        for pk in BIG[:alpha]:
            rk = float(rng.choice(((pk - 1) // 2, -((pk - 1) // 2))))
            hat = float(rng.randrange(-(qi // 2), qi // 2))
            acc = _add(acc, mulm(rk, hat, qi))
            exact += int(rk) * int(hat)
        assert abs(acc) < LIM
        assert (int(redm(acc, qi)) - exact) % qi == 0


def test_big_primes_are_the_ring_primes():
    """BIG holds primes 1 (mod 2^16) below 2^50, checked by trial division
    against every prime below 2^13 and a Fermat test in two bases."""
    for p in BIG:
        assert p < 1 << 50 and (p - 1) % (1 << 16) == 0
        assert all(pow(b, p - 1, p) == 1 for b in (2, 3))
        assert all(p % d for d in range(3, 1 << 13, 2))
