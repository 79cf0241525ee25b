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

Q = 1125899906826241          # a 50-bit NTT prime, 1 (mod 2^15)
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


def mulm(a: float, b: float) -> float:
    h = a * b                                   # rounded product
    l = float(int(a) * int(b) - int(h))         # its exact error (fma(a, b, -h))
    assert abs(l) < LIM
    e = _rint(h * QI)
    r = _fma_exact(-e, Q, h)
    return _add(r, l)


def redm(x: float) -> float:
    assert abs(x) < LIM
    return _fma_exact(-_rint(x * QI), Q, x)


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


def inverse(x, tw, exact):
    """Gentleman-Sande stages, stage g pairs i and i + 2^g with twiddle
    tw[n / 2^(g+1) + block]."""
    n = len(x)
    logn = n.bit_length() - 1
    worst = 0
    for g in range(logn):
        d = 1 << g
        red = (g & 1) or g == logn - 1
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
