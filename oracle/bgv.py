"""Oracle BGV layer: keys, encryption, decryption and the HE primitives.

Test infrastructure only; shares no code with the GPU library.

Ciphertexts are lists of components, each an (L, N) uint64 array in
coefficient form with residues in [0, q_i) (the canonical form).  Products are
formed through the oracle's own transform (checked against the schoolbook
product in the tests).  Decryption uses exact big-integer CRT.

HE primitives follow the paper's Section II-A set: HE-Add, HE-Mult (ct x ct),
HE-CMult (ct x plaintext) and HE-Rot (left rotation by i slots).  The
linear-transform building block is the diagonal method of Section III-B-1:
sum over diagonals z of u_z (.) Rot(m, z).
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import ring
from .ring import Params

Ct = List[np.ndarray]


class SecretKey:
    def __init__(self, P: Params, master: int):
        self.P = P
        self.master = master
        s0 = ring.stream_seed(master, ring.TAG_SECRET, 0)
        self.s = ring.sample_ternary(s0, 0, P.N)            # signed coefficients
        self.s_ext = ring.reduce_signed(self.s, P.ext_arr)  # rows over the extended basis


class SwitchKey:
    """Key switching from s' to s: per digit j a pair (b_j, a_j) over the
    extended basis, kept in the oracle's evaluation form.

    a_j is sampled directly in the evaluation domain: its value at
    psi_r^(2i+1) (prime r of the extended basis, natural index i, psi_r the
    root of ring.primitive_2n_root) is the uniform draw r*N + i of the digit's
    stream.  The evaluations of a uniform polynomial are uniform, so this is
    the same distribution as sampling coefficients; it lets an evaluator
    regenerate a_j from the stream instead of storing it.  The error e_j is
    sampled in coefficient form (draws from nExt*N on) as before."""

    def __init__(self, P: Params, sk: SecretKey, s_prime_ext: np.ndarray, tag: int, idx_base: int):
        self.digits = []
        mod, psi = P.ext_arr, P.psi_ext
        s_eval = ring.ntt(sk.s_ext, mod, psi)
        sp_eval = ring.ntt(s_prime_ext, mod, psi)
        nrow = P.L + P.alpha
        for j, (d0, d1) in enumerate(P.digits):
            s0 = ring.stream_seed(sk.master, tag, idx_base + j)
            a_eval = ring.sample_uniform(s0, 0, mod, P.N)   # evaluation form, natural order
            e = ring.sample_gauss(P, s0, nrow * P.N)
            # gadget factor: [P]_{q_i} on the digit's own primes, 0 elsewhere
            gadget = [(P.P % P.ext[r]) if d0 <= r < d1 else 0 for r in range(nrow)]
            te = ring.reduce_signed(e * P.t, mod)
            te_eval = ring.ntt(te, mod, psi)
            b_eval = ring.sub(te_eval, ring.mul(a_eval, s_eval, mod), mod)
            b_eval = ring.add(b_eval, ring.scale(sp_eval, gadget, mod), mod)
            self.digits.append((b_eval, a_eval))


class KeySet:
    def __init__(self, P: Params, master: int, galois_elements: Sequence[int] = (), relin: bool = True):
        self.P = P
        self.sk = SecretKey(P, master)
        self.rot: Dict[int, SwitchKey] = {}
        self.relin: Optional[SwitchKey] = None
        if relin:
            s2 = ring.polymul(P, self.sk.s_ext, self.sk.s_ext)
            self.relin = SwitchKey(P, self.sk, s2, ring.TAG_RELIN, 0)
        for g in sorted(set(galois_elements)):
            self.add_rotation(g)

    def add_rotation(self, g: int):
        P = self.P
        if g in self.rot or g == 1:
            return
        s_g = ring.automorph(self.sk.s_ext, g, P.ext_arr)
        self.rot[g] = SwitchKey(P, self.sk, s_g, ring.TAG_ROT, g * 256)


# ---------------------------------------------------------------------------
# encryption / decryption
# ---------------------------------------------------------------------------

def enc_stream_index(role: int, block: int, nonce: int) -> int:
    return (nonce * 4096 + block * 4 + role) % 2**64


def encrypt_poly(ks: KeySet, mu: np.ndarray, role: int, block: int, nonce: int) -> Ct:
    """Secret-key RLWE encryption of the plaintext polynomial mu (coefficients
    in [0, t)): c1 = a, c0 = -a*s + t*e + lift(mu)."""
    P = ks.P
    s0 = ring.stream_seed(ks.sk.master, ring.TAG_ENC, enc_stream_index(role, block, nonce))
    a = ring.sample_uniform(s0, 0, P.q_arr, P.N)
    e = ring.sample_gauss(P, s0, P.L * P.N)
    m_signed = ring.lift_centered(mu, P.t)
    noisy = ring.reduce_signed(e * P.t + m_signed, P.q_arr)
    s_q = ks.sk.s_ext[:P.L]
    c0 = ring.sub(noisy, ring.polymul(P, a, s_q), P.q_arr)
    return [c0, a]


def encrypt_slots(ks: KeySet, slots: Sequence[int], role: int = 2, block: int = 0, nonce: int = 0) -> Ct:
    return encrypt_poly(ks, ring.encode(ks.P, slots), role, block, nonce)


def _combine(ks: KeySet, ct: Ct) -> np.ndarray:
    """c0 + c1 s (+ c2 s^2) over the ciphertext's primes (its level: the
    first rows of Q; fewer than L after modulus switching)."""
    P = ks.P
    lv = ct[0].shape[0]
    s_q = ks.sk.s_ext[:lv]
    acc = ct[0]
    spow = s_q
    for comp in ct[1:]:
        acc = ring.add(acc, ring.polymul(P, comp, spow), P.q_arr[:lv])
        spow = ring.polymul(P, spow, s_q)
    return acc


def decrypt_poly(ks: KeySet, ct: Ct) -> np.ndarray:
    """c0 + c1 s (+ c2 s^2) over Q -> exact CRT -> centered -> mod t."""
    return crt_centered_mod_t(ks.P, _combine(ks, ct))


def crt_centered_mod_t(P: Params, rows: np.ndarray) -> np.ndarray:
    """Residues over Q (or the first rows of it) -> the integer in (-Q/2, Q/2)
    -> reduced mod t."""
    qs = P.q[: rows.shape[0]]
    Q = math.prod(qs)
    basis = []
    for qi in qs:
        hat = Q // qi
        basis.append(hat * pow(hat % qi, -1, qi))
    out = np.empty(P.N, dtype=np.int64)
    cols = [[int(v) for v in rows[i]] for i in range(len(qs))]
    for k in range(P.N):
        x = 0
        for i in range(len(qs)):
            x += cols[i][k] * basis[i]
        x %= Q
        if x > Q // 2:
            x -= Q
        out[k] = x % P.t
    return out


def noise_bits(ks: KeySet, ct: Ct, mu: np.ndarray) -> float:
    """log2 of the largest |c0 + c1 s - lift(mu)| over coefficients (a diagnostic)."""
    P = ks.P
    acc = _combine(ks, ct)
    qs = P.q[: acc.shape[0]]
    Q = math.prod(qs)
    basis = [(Q // qi) * pow((Q // qi) % qi, -1, qi) for qi in qs]
    worst = 0
    lifted = ring.lift_centered(mu, P.t)
    for k in range(P.N):
        x = sum(int(acc[i][k]) * basis[i] for i in range(len(qs))) % Q
        if x > Q // 2:
            x -= Q
        worst = max(worst, abs(x - int(lifted[k])))
    return math.log2(worst) if worst else 0.0


def decrypt_slots(ks: KeySet, ct: Ct) -> List[int]:
    return ring.decode(ks.P, decrypt_poly(ks, ct))


# ---------------------------------------------------------------------------
# primitives
# ---------------------------------------------------------------------------

def he_add(P: Params, a: Ct, b: Ct) -> Ct:
    n = max(len(a), len(b))
    out = []
    for i in range(n):
        if i < len(a) and i < len(b):
            out.append(ring.add(a[i], b[i], P.q_arr))
        else:
            out.append((a[i] if i < len(a) else b[i]).copy())
    return out


def tensor(P: Params, a: Ct, b: Ct) -> Ct:
    """(a0, a1) x (b0, b1) -> (a0 b0, a0 b1 + a1 b0, a1 b1)."""
    a0, a1 = a
    b0, b1 = b
    c0 = ring.polymul(P, a0, b0)
    c1 = ring.add(ring.polymul(P, a0, b1), ring.polymul(P, a1, b0), P.q_arr)
    c2 = ring.polymul(P, a1, b1)
    return [c0, c1, c2]


def ks_inner(P: Params, c: np.ndarray, key: SwitchKey) -> Tuple[np.ndarray, np.ndarray]:
    """u = sum_j ModUp_j(c) * (b_j, a_j) over the extended basis, returned in
    the oracle's evaluation form."""
    mod, psi = P.ext_arr, P.psi_ext
    u0 = np.zeros((P.L + P.alpha, P.N), dtype=np.uint64)
    u1 = np.zeros_like(u0)
    for j in range(P.beta):
        y = ring.ntt(ring.modup_digit(P, c, j), mod, psi)
        b, a = key.digits[j]
        u0 = ring.add(u0, ring.mul(y, b, mod), mod)
        u1 = ring.add(u1, ring.mul(y, a, mod), mod)
    return u0, u1


def moddown_eval(P: Params, u_eval: np.ndarray) -> np.ndarray:
    return ring.moddown(P, ring.intt(u_eval, P.ext_arr, P.psi_ext))


class Mask:
    """A 0/1 slot vector as a plaintext polynomial: its centered lift reduced
    over the extended basis, in the oracle's evaluation form."""

    def __init__(self, P: Params, slots: Sequence[int]):
        self.slots = list(slots)
        mu = ring.encode(P, self.slots)
        self.lift = ring.lift_centered(mu, P.t)
        self.ext_eval = ring.ntt(ring.reduce_signed(self.lift, P.ext_arr), P.ext_arr, P.psi_ext)
        self.q_eval = self.ext_eval[:P.L]


def rot_sum(P: Params, ks: KeySet, ct: Ct, terms: Sequence[Tuple[int, Optional[Mask]]]) -> Ct:
    """sum over terms (z, mask) of mask (.) Rot(ct, z), with one shared division
    by P for all key-switched terms (mask None: no multiply).

      out0 = sum mask . phi_z(c0)              + ModDown(sum_{z != 0} mask . u_{z,0})
      out1 = sum_{z = 0 mod S} mask . c1       + ModDown(sum_{z != 0} mask . u_{z,1})

    where u_z is the key-switching inner product of phi_z(c1) under the key
    for phi_z(s).  ModDown is applied only if some term needs a key switch.
    A single term (0, None) is the identity."""
    assert len(ct) == 2
    c0, c1 = ct
    L = P.L
    qm, qpsi = P.q_arr, P.psi_q
    ext, epsi = P.ext_arr, P.psi_ext
    out0 = np.zeros((L, P.N), dtype=np.uint64)   # evaluation form
    out1 = np.zeros_like(out0)
    U0 = np.zeros((L + P.alpha, P.N), dtype=np.uint64)
    U1 = np.zeros_like(U0)
    switched = False
    c0e = ring.ntt(c0, qm, qpsi)
    c1e = ring.ntt(c1, qm, qpsi)
    for z, mask in terms:
        zz = z % P.S
        if zz == 0:
            if mask is None:
                out0 = ring.add(out0, c0e, qm)
                out1 = ring.add(out1, c1e, qm)
            else:
                out0 = ring.add(out0, ring.mul(c0e, mask.q_eval, qm), qm)
                out1 = ring.add(out1, ring.mul(c1e, mask.q_eval, qm), qm)
            continue
        g = P.galois(zz)
        if g not in ks.rot:
            raise KeyError(f"no rotation key for z={z} (g={g})")
        c0g = ring.ntt(ring.automorph(c0, g, qm), qm, qpsi)
        u0, u1 = ks_inner(P, ring.automorph(c1, g, qm), ks.rot[g])
        if mask is not None:
            c0g = ring.mul(c0g, mask.q_eval, qm)
            u0 = ring.mul(u0, mask.ext_eval, ext)
            u1 = ring.mul(u1, mask.ext_eval, ext)
        out0 = ring.add(out0, c0g, qm)
        U0 = ring.add(U0, u0, ext)
        U1 = ring.add(U1, u1, ext)
        switched = True
    r0 = ring.intt(out0, qm, qpsi)
    r1 = ring.intt(out1, qm, qpsi)
    if switched:
        r0 = ring.add(r0, moddown_eval(P, U0), qm)
        r1 = ring.add(r1, moddown_eval(P, U1), qm)
    return [r0, r1]


def rotate(P: Params, ks: KeySet, ct: Ct, z: int) -> Ct:
    """HE-Rot(ct, z) of Section II-A: left rotation of the row-0 slots by z
    (negative: right).  With g = 5^(z mod S) mod 2N:

      (phi_g(c0) + ModDown(u0), ModDown(u1)),  u = inner product of ModUp(phi_g(c1))
                                                with the key for phi_g(s),

    one division by P per rotation.  z = 0 (mod S) is the identity."""
    assert len(ct) == 2
    zz = z % P.S
    if zz == 0:
        return [c.copy() for c in ct]
    g = P.galois(zz)
    if g not in ks.rot:
        raise KeyError(f"no rotation key for z={z} (g={g})")
    c0, c1 = ct
    u0, u1 = ks_inner(P, ring.automorph(c1, g, P.q_arr), ks.rot[g])
    return [ring.add(ring.automorph(c0, g, P.q_arr), moddown_eval(P, u0), P.q_arr),
            moddown_eval(P, u1)]


def lin_transform(P: Params, ks: KeySet, ct: Ct, terms: Sequence[Tuple[int, Optional[Mask]]]) -> Ct:
    """The diagonal method of Section III-B-1, Eq. (lintrans), in the paper's
    own primitive order: for every nonzero diagonal z one complete HE-Rot
    (its own division by P), then HE-CMult by the diagonal's mask u_z, then
    HE-Add into the sum.  A term with mask None is added unmasked.

    Decrypts to the same slots as rot_sum; the ciphertext bits differ, because
    here each rotation is divided by P before its mask multiplies it."""
    out = None
    for z, mask in terms:
        r = rotate(P, ks, ct, z)
        if mask is not None:
            r = he_cmult(P, r, mask)
        out = r if out is None else he_add(P, out, r)
    return out


def relinearize(P: Params, ks: KeySet, ct: Ct) -> Ct:
    """(c0, c1, c2) -> (c0 + ModDown(u0), c1 + ModDown(u1)), u the inner
    product of ModUp(c2) with the key for s^2."""
    c0, c1, c2 = ct
    u0, u1 = ks_inner(P, c2, ks.relin)
    return [ring.add(c0, moddown_eval(P, u0), P.q_arr),
            ring.add(c1, moddown_eval(P, u1), P.q_arr)]


def he_mult(P: Params, ks: KeySet, a: Ct, b: Ct) -> Ct:
    """HE-Mult: tensor then relinearise."""
    return relinearize(P, ks, tensor(P, a, b))


def he_cmult(P: Params, ct: Ct, mask: Mask) -> Ct:
    """HE-CMult by a plaintext slot vector."""
    return [ring.intt(ring.mul(ring.ntt(c, P.q_arr, P.psi_q), mask.q_eval, P.q_arr), P.q_arr, P.psi_q)
            for c in ct]


def mod_switch(P: Params, ct: Ct, drop: int = 1) -> Ct:
    """BGV modulus switching: drop the last `drop` primes of the ciphertext
    (coefficient form), one at a time, keeping the plaintext.

    From level l (primes q_0..q_{l-1}) to l - 1, with q = q_{l-1} and
    k = q mod t: each component, read as the integer x in [0, Q_l), becomes
    y = k x mod Q_l, then z = (y - delta) / q with delta = t [y t^-1]_q
    (centered), so that delta = y (mod q) and delta = 0 (mod t) and the
    division is exact; z is reduced mod q_0..q_{l-2}.  Decryption then gives
    k mu q^-1 = mu (mod t), and the noise becomes about k/q of what it was
    plus t (1 + |s|_1) / 2 (the standard rescaling of BGV; the factor k keeps
    the plaintext unscaled)."""
    out = [np.ascontiguousarray(c, dtype=np.uint64) for c in ct]
    if drop < 1 or drop >= out[0].shape[0]:
        raise ValueError("drop must leave at least one prime")
    for _ in range(drop):
        lv = out[0].shape[0]
        qs = P.q[:lv]
        q = qs[-1]
        Q = math.prod(qs)
        k = q % P.t
        tinv = pow(P.t, -1, q)
        basis = [(Q // qi) * pow((Q // qi) % qi, -1, qi) for qi in qs]
        nxt = []
        for c in out:
            cols = [[int(v) for v in c[i]] for i in range(lv)]
            rows = np.empty((lv - 1, P.N), dtype=np.uint64)
            for j in range(P.N):
                x = sum(cols[i][j] * basis[i] for i in range(lv)) % Q
                y = (k * x) % Q
                r = (y * tinv) % q
                if r > q // 2:
                    r -= q
                num = y - P.t * r
                assert num % q == 0
                z = num // q
                for i in range(lv - 1):
                    rows[i, j] = z % qs[i]
            nxt.append(rows)
        out = nxt
    return out
