"""Oracle ring layer: parameters, transforms, sampling and slot encoding.

Test infrastructure: only tests, the smoke check and the benchmark's CPU
baseline use this package.  Nothing here is shared with the GPU library.

The ring is R_q = Z_q[X]/(X^N + 1) (Section IV-A of the paper), held in RNS
form: one row of N residues per prime.
"""
from __future__ import annotations

import ctypes
import functools
from decimal import Decimal, getcontext
from typing import List, Sequence

import numpy as np

from . import build as _build

_lib = ctypes.CDLL(_build.build())
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_U64 = ctypes.c_uint64
_I = ctypes.c_int

_lib.or_ntt_rows.argtypes = [_u64p, _I, _I, _u64p, _u64p]
_lib.or_intt_rows.argtypes = [_u64p, _I, _I, _u64p, _u64p]
_lib.or_negacyclic_schoolbook.argtypes = [_u64p, _u64p, _u64p, _I, _U64]
for _name in ("or_mul_rows", "or_add_rows", "or_sub_rows", "or_scale_rows"):
    getattr(_lib, _name).argtypes = [_u64p, _u64p, _u64p, _I, _I, _u64p]
_lib.or_reduce_signed_rows.argtypes = [_u64p, _i64p, _I, _I, _u64p]
_lib.or_automorph_rows.argtypes = [_u64p, _u64p, _I, _I, _u64p, _U64]
_lib.or_mix64.argtypes = [_U64]
_lib.or_mix64.restype = _U64
_lib.or_stream_seed.argtypes = [_U64, _U64, _U64]
_lib.or_stream_seed.restype = _U64
_lib.or_sample_uniform.argtypes = [_u64p, _U64, _U64, _I, _I, _u64p]
_lib.or_sample_ternary.argtypes = [_i64p, _U64, _U64, _I]
_lib.or_sample_cdt.argtypes = [_i64p, _U64, _U64, _I, _u64p, _I, ctypes.c_int64]
_lib.or_modup_digit.argtypes = [_u64p, _u64p, _I, _I, _I, _u64p, _I, _I]
_lib.or_moddown.argtypes = [_u64p, _u64p, _I, _I, _I, _u64p, _U64]

SIGMA = Decimal("3.2")
GAUSS_BOUND = 19          # support of the error distribution is [-19, 19]
PRIME_BITS = 50


# ---------------------------------------------------------------------------
# number theory helpers (plain Python integers)
# ---------------------------------------------------------------------------

def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin for n < 3.3e24 (first 12 prime bases)."""
    if n < 2:
        return False
    small = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)
    for p in small:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def ntt_primes(N: int, count: int, bits: int = PRIME_BITS) -> List[int]:
    """The first `count` primes below 2^bits that are 1 mod 2N, descending."""
    out = []
    k = ((1 << bits) - 2) // (2 * N)
    while len(out) < count:
        p = k * 2 * N + 1
        if p < (1 << bits) and is_prime(p):
            out.append(p)
        k -= 1
    return out


def primitive_2n_root(q: int, N: int) -> int:
    """Some psi with psi^N = -1 (mod q): the first x^((q-1)/2N), x = 2, 3, ..., that works."""
    e = (q - 1) // (2 * N)
    x = 2
    while True:
        w = pow(x, e, q)
        if pow(w, N, q) == q - 1:
            return w
        x += 1


def smallest_2n_root(t: int, N: int) -> int:
    """zeta_t: the smallest x in [2, t) with x^N = -1 (mod t)."""
    for x in range(2, t):
        if pow(x, N, t) == t - 1:
            return x
    raise ValueError("no primitive 2N-th root of unity mod t")


@functools.lru_cache(maxsize=None)
def gaussian_cdt() -> tuple:
    """T[k] = floor(2^64 * F(-19 + k)), k = 0..37, F the CDF of the discrete
    Gaussian rho(x) = exp(-x^2 / (2 sigma^2)) restricted to [-19, 19]."""
    getcontext().prec = 80
    xs = range(-GAUSS_BOUND, GAUSS_BOUND + 1)
    rho = [(-(Decimal(x) ** 2) / (2 * SIGMA * SIGMA)).exp() for x in xs]
    z = sum(rho)
    out, acc = [], Decimal(0)
    for k in range(2 * GAUSS_BOUND):
        acc += rho[k]
        out.append(int((acc / z) * (Decimal(2) ** 64)))
    return tuple(out)


# ---------------------------------------------------------------------------
# parameters
# ---------------------------------------------------------------------------

class Params:
    """Primes, roots and basis constants of one parameter set.

    Extended basis order: q_0..q_{L-1} then p_0..p_{alpha-1}.  The special
    primes p are the alpha largest; the ciphertext primes q follow in
    descending order.
    """

    def __init__(self, N: int, t: int, L: int, alpha: int, prime_bits: int = PRIME_BITS):
        assert N & (N - 1) == 0 and N >= 4
        assert (t - 1) % (2 * N) == 0 and is_prime(t)
        self.N, self.t, self.L, self.alpha = N, t, L, alpha
        self.prime_bits = prime_bits
        self.S = N // 2
        primes = ntt_primes(N, L + alpha, prime_bits)
        self.p = primes[:alpha]
        self.q = primes[alpha:]
        self.ext = self.q + self.p
        self.Q = 1
        for x in self.q:
            self.Q *= x
        self.P = 1
        for x in self.p:
            self.P *= x
        self.psi = [primitive_2n_root(x, N) for x in self.ext]
        self.zeta = smallest_2n_root(t, N)
        self.psi_t = self.zeta
        # digits of alpha consecutive q primes: [(d0, d1), ...]
        self.digits = [(j, min(j + alpha, L)) for j in range(0, L, alpha)]
        self.beta = len(self.digits)
        self.q_arr = np.array(self.q, dtype=np.uint64)
        self.ext_arr = np.array(self.ext, dtype=np.uint64)
        self.psi_q = np.array(self.psi[:L], dtype=np.uint64)
        self.psi_ext = np.array(self.psi, dtype=np.uint64)
        self.cdt = np.array(gaussian_cdt(), dtype=np.uint64)
        # slot s of row 0 sits at exponent 5^s mod 2N, row 1 at -5^s mod 2N
        self.slot_exp = [pow(5, s, 2 * N) for s in range(self.S)]

    def galois(self, z: int) -> int:
        """Galois element of a left rotation by z slots: 5^(z mod S) mod 2N."""
        return pow(5, z % self.S, 2 * self.N)

    def moduli(self, rows: int) -> np.ndarray:
        return self.q_arr if rows == self.L else self.ext_arr


# ---------------------------------------------------------------------------
# row-wise polynomial operations (arrays of shape (rows, N), uint64)
# ---------------------------------------------------------------------------

def _rows(a: np.ndarray):
    return a.shape[0], a.shape[1]


def ntt(a: np.ndarray, mod: np.ndarray, psi: np.ndarray) -> np.ndarray:
    out = np.ascontiguousarray(a, dtype=np.uint64).copy()
    r, n = _rows(out)
    _lib.or_ntt_rows(out, r, n, np.ascontiguousarray(mod[:r]), np.ascontiguousarray(psi[:r]))
    return out


def intt(a: np.ndarray, mod: np.ndarray, psi: np.ndarray) -> np.ndarray:
    out = np.ascontiguousarray(a, dtype=np.uint64).copy()
    r, n = _rows(out)
    _lib.or_intt_rows(out, r, n, np.ascontiguousarray(mod[:r]), np.ascontiguousarray(psi[:r]))
    return out


def _binop(fn, a, b, mod):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    out = np.empty_like(a)
    r, n = _rows(a)
    fn(out, a, b, r, n, np.ascontiguousarray(mod[:r]))
    return out


def mul(a, b, mod):
    return _binop(_lib.or_mul_rows, a, b, mod)


def add(a, b, mod):
    return _binop(_lib.or_add_rows, a, b, mod)


def sub(a, b, mod):
    return _binop(_lib.or_sub_rows, a, b, mod)


def scale(a, consts: Sequence[int], mod):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    out = np.empty_like(a)
    r, n = _rows(a)
    c = np.array([int(x) % int(mod[i]) for i, x in enumerate(consts[:r])], dtype=np.uint64)
    _lib.or_scale_rows(out, a, c, r, n, np.ascontiguousarray(mod[:r]))
    return out


def reduce_signed(x: np.ndarray, mod: np.ndarray) -> np.ndarray:
    """Signed integer polynomial (int64, length N) -> rows of residues."""
    x = np.ascontiguousarray(x, dtype=np.int64)
    out = np.empty((len(mod), x.shape[0]), dtype=np.uint64)
    _lib.or_reduce_signed_rows(out, x, len(mod), x.shape[0], np.ascontiguousarray(mod))
    return out


def automorph(a: np.ndarray, g: int, mod: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    out = np.empty_like(a)
    r, n = _rows(a)
    _lib.or_automorph_rows(out, a, r, n, np.ascontiguousarray(mod[:r]), g)
    return out


def polymul(P: Params, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Product in R_q (coefficient form in, coefficient form out)."""
    r = a.shape[0]
    mod = P.moduli(r)
    psi = P.psi_ext[:r]
    return intt(mul(ntt(a, mod, psi), ntt(b, mod, psi), mod), mod, psi)


def schoolbook(a: np.ndarray, b: np.ndarray, q: int) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    out = np.empty_like(a)
    _lib.or_negacyclic_schoolbook(out, a, b, a.shape[0], q)
    return out


# ---------------------------------------------------------------------------
# random streams
# ---------------------------------------------------------------------------

TAG_SECRET, TAG_RELIN, TAG_ROT, TAG_ENC = 1, 2, 3, 4


def mix64(z: int) -> int:
    return int(_lib.or_mix64(z & (2**64 - 1)))


def stream_seed(master: int, tag: int, idx: int) -> int:
    return int(_lib.or_stream_seed(master & (2**64 - 1), tag, idx & (2**64 - 1)))


def sample_uniform(s0: int, first: int, mod: np.ndarray, N: int) -> np.ndarray:
    out = np.empty((len(mod), N), dtype=np.uint64)
    _lib.or_sample_uniform(out, s0, first, len(mod), N, np.ascontiguousarray(mod))
    return out


def sample_ternary(s0: int, first: int, N: int) -> np.ndarray:
    out = np.empty(N, dtype=np.int64)
    _lib.or_sample_ternary(out, s0, first, N)
    return out


def sample_gauss(P: Params, s0: int, first: int) -> np.ndarray:
    out = np.empty(P.N, dtype=np.int64)
    _lib.or_sample_cdt(out, s0, first, P.N, P.cdt, len(P.cdt), -GAUSS_BOUND)
    return out


# ---------------------------------------------------------------------------
# slot encoding (SIMD packing of Smart-Vercauteren, the paper's Section II-A)
# ---------------------------------------------------------------------------

def _t_arr(P: Params):
    return np.array([P.t], dtype=np.uint64), np.array([P.zeta], dtype=np.uint64)


def encode(P: Params, slots: Sequence[int], row1: Sequence[int] = None) -> np.ndarray:
    """Slot vector (row 0, S values mod t; row 1 zero unless given) -> the
    unique polynomial mu of degree < N over Z_t with mu(zeta^(5^s)) = slot s
    (row 0) and mu(zeta^(-5^s)) = row-1 slot s.  Returns int64 coefficients
    in [0, t)."""
    N, t = P.N, P.t
    ev = np.zeros((1, N), dtype=np.uint64)
    for s in range(P.S):
        e = P.slot_exp[s]
        ev[0, (e - 1) // 2] = int(slots[s]) % t if s < len(slots) else 0
        e1 = 2 * N - e
        ev[0, (e1 - 1) // 2] = (int(row1[s]) % t) if row1 is not None and s < len(row1) else 0
    tq, tz = _t_arr(P)
    return intt(ev, tq, tz)[0].astype(np.int64)


def decode(P: Params, mu: np.ndarray, both_rows: bool = False):
    """Inverse of encode: evaluate mu (coefficients mod t) at the slot points."""
    tq, tz = _t_arr(P)
    ev = ntt(np.array([[int(x) % P.t for x in mu]], dtype=np.uint64), tq, tz)[0]
    row0 = [int(ev[(e - 1) // 2]) for e in P.slot_exp]
    if not both_rows:
        return row0
    row1 = [int(ev[(2 * P.N - e - 1) // 2]) for e in P.slot_exp]
    return row0, row1


def lift_centered(mu: np.ndarray, t: int) -> np.ndarray:
    """[0, t) -> (-t/2, t/2]: v stays if v <= (t-1)/2, else v - t."""
    mu = np.asarray(mu, dtype=np.int64)
    return np.where(mu > (t - 1) // 2, mu - t, mu)


def modup_digit(P: Params, c: np.ndarray, j: int) -> np.ndarray:
    """Digit j of c (coefficient form over Q) lifted to the extended basis."""
    d0, d1 = P.digits[j]
    c = np.ascontiguousarray(c, dtype=np.uint64)
    y = np.empty((P.L + P.alpha, P.N), dtype=np.uint64)
    _lib.or_modup_digit(y, c, P.N, P.L, P.alpha, P.ext_arr, d0, d1)
    return y


def moddown(P: Params, u: np.ndarray) -> np.ndarray:
    """Coefficient-form extended-basis polynomial -> divided by P over Q."""
    u = np.ascontiguousarray(u, dtype=np.uint64)
    out = np.empty((P.L, P.N), dtype=np.uint64)
    _lib.or_moddown(out, u, P.N, P.L, P.alpha, P.ext_arr, P.t)
    return out
