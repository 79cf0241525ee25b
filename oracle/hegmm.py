"""Oracle HEGMM-En: planning, client packing, the cloud-side loop, unpacking.

Test infrastructure only; shares no code with the GPU library.

Follows Algorithm 2 (HEGMM-Enhanced) of the paper (Section III-C) built on the
element-wise identity of Section III-A:

    A.B = sum_{k<l} (eps^k o sigma(A)) (.) (omega^k o tau(B)),

with the operand duplication of Theorems 5/6, column-major flattening, and the
linear transforms realised by the diagonal method (Section III-B-1).  Readings
where the paper is silent (layout of the result, removal of redundant partial
products, when to relinearise, what to do when the operands do not fit one
ciphertext) are the ones listed in the design notes and restated at each
function below.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import bgv, ring
from .ring import Params


# ---------------------------------------------------------------------------
# planning
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Plan:
    m: int                 # original shape
    l: int
    n: int
    transposed: bool       # solve B^T A^T instead (the p == n branch of Algorithm 2)
    mo: int                # oriented problem: X (mo x l) times Y (l x no)
    no: int
    nb: int                # number of inner-dimension blocks (1 if the operands fit)
    lb: int                # inner block length (zero padded)
    d: int                 # duplication count of X (Theorem 5)
    M: int                 # rows of the duplicated X, the column stride of the layout
    K: int                 # loop trips
    W: int                 # packed width of the left operand
    eps: List[List[Tuple[int, Optional[frozenset]]]]    # per k: (z, mask slots or None)
    omega: List[List[Tuple[int, Optional[frozenset]]]]
    fold: List[int]        # rotation amounts summed after relinearisation (0 first)
    method: int = 2        # 2: HEGMM-En (Algorithm 2); 1: HEGMM (Algorithm 1); 3: Algorithm 1, sigma/tau in the cloud
    sigma: List[Tuple[int, Optional[frozenset]]] = dataclasses.field(default_factory=list)   # method 3
    tau: List[Tuple[int, Optional[frozenset]]] = dataclasses.field(default_factory=list)

    def rotations(self, S: int) -> List[int]:
        zs = set()
        for terms in self.eps + self.omega + [self.sigma, self.tau]:
            for z, _ in terms:
                if z % S:
                    zs.add(z % S)
        for z in self.fold:
            if z % S:
                zs.add(z % S)
        return sorted(zs)


def _constants(mo: int, lb: int, no: int):
    d = -(-lb // mo) if mo < lb else 1
    M = d * mo
    K = min(mo, lb)
    W = max(lb, no)
    return d, M, K, W


def orientation(m: int, l: int, n: int) -> bool:
    """Transpose iff n is the strict smallest of (m, n) among the minima,
    following Algorithm 2's if-order: p == m first, then p == n, else l."""
    p = min(m, l, n)
    if p == m:
        return False
    return p == n


def plan(m: int, l: int, n: int, S: int, method: int = 2, min_blocks: int = 1) -> Plan:
    if min(m, l, n) <= 0:
        raise ValueError("dimensions must be positive")
    if method in (1, 3):
        if min_blocks > 1:
            raise ValueError("forced blocking needs HEGMM-En")
        return plan_alg1(m, l, n, S, cloud=method == 3)
    tr = orientation(m, l, n)
    mo, no = (n, m) if tr else (m, n)

    def fits(lb):
        d, M, K, W = _constants(mo, lb, no)
        return M * W <= S

    # Section IV-D: when the operands do not fit one ciphertext, split the
    # inner dimension into the fewest blocks that fit (at least min_blocks,
    # to force the blockwise product on shapes that would fit whole), each
    # block product accumulated into the same result
    nb = min(max(min_blocks, 1), l)
    while nb <= l and not fits(-(-l // nb)):
        nb += 1
    if nb > l:
        raise ValueError("shape does not fit one ciphertext even with inner blocking")
    lb = -(-l // nb)
    d, M, K, W = _constants(mo, lb, no)
    region = frozenset(i + j * M for i in range(M) for j in range(no))

    eps, omega = [], []
    for k in range(K):
        eps.append(_terms(eps_diagonals(mo, lb, no, M, W, k), region, [k * M, (k - lb) * M]))
        omega.append(_terms(omega_diagonals(lb, no, M, k), region, [k, k - lb]))
    fold = [h * mo for h in range(d)]
    return Plan(m, l, n, tr, mo, no, nb, lb, d, M, K, W, eps, omega, fold)


def alg1_eps_diagonals(mo: int, l: int, no: int, k: int) -> Dict[int, set]:
    """Algorithm 1's eps^k_{mo x no} on sigma(X) flattened column-major
    (mo x l, column stride mo): output (i, j) reads column (j + k) mod l,
    i.e. slot i + ((j + k) mod l) mo, a left rotation by the difference."""
    cand: Dict[int, set] = {}
    for i in range(mo):
        for j in range(no):
            src = i + ((j + k) % l) * mo
            cand.setdefault(src - (i + j * mo), set()).add(i + j * mo)
    return cand


def alg1_omega_diagonals(mo: int, l: int, no: int, k: int) -> Dict[int, set]:
    """Algorithm 1's omega^k_{mo x no} on tau(Y) flattened column-major
    (l x no, column stride l): output (i, j) reads row (i + k) mod l of
    column j, i.e. slot ((i + k) mod l) + j l."""
    cand: Dict[int, set] = {}
    for i in range(mo):
        for j in range(no):
            src = ((i + k) % l) + j * l
            cand.setdefault(src - (i + j * mo), set()).add(i + j * mo)
    return cand


def _alg1_count(mo: int, l: int, no: int, S: int) -> int:
    c = 0
    for k in range(l):
        for cand in (alg1_eps_diagonals(mo, l, no, k), alg1_omega_diagonals(mo, l, no, k)):
            c += sum(1 for z in cand if z % S)
    return c


def sigma_diagonals(mo: int, l: int) -> Dict[int, set]:
    """sigma on X (mo x l) flattened column-major (Section III-A definition
    sigma(X)[i][j] = X[i][(i + j) mod l]): output slot i + j mo reads slot
    i + ((i + j) mod l) mo, a left rotation by the difference."""
    cand: Dict[int, set] = {}
    for i in range(mo):
        for j in range(l):
            dst = i + j * mo
            cand.setdefault(i + ((i + j) % l) * mo - dst, set()).add(dst)
    return cand


def tau_diagonals(l: int, no: int) -> Dict[int, set]:
    """tau on Y (l x no) flattened column-major (tau(Y)[i][j] =
    Y[(i + j) mod l][j]): output slot i + j l reads slot ((i + j) mod l) + j l."""
    cand: Dict[int, set] = {}
    for i in range(l):
        for j in range(no):
            dst = i + j * l
            cand.setdefault(((i + j) % l) + j * l - dst, set()).add(dst)
    return cand


def plan_alg1(m: int, l: int, n: int, S: int, cloud: bool = False) -> Plan:
    """Algorithm 1 (HEGMM): C = sum_{k<l} eps^k(sigma(A)) (.) omega^k(tau(B)),
    sigma and tau applied by the client while packing (as in the paper's
    experiments), matrices flattened column-major -- or row-major, i.e. the
    transposed problem B^T A^T column-major, when that needs fewer
    key-switched diagonals in total (ties: column-major).  No duplication, so
    d = 1 and no fold; the result sits at slot i + j m (j + i n transposed).
    Needs max(m l, l n, m n) <= S.

    cloud=True (method 3): the client packs X and Y as they are (column-major)
    and the cloud applies sigma and tau to the ciphertexts as linear
    transforms by the diagonal method, with the 2 min(mo, l) - 1 and
    2 min(no, l) - 1 diagonals of Theorems 1 and 2, before the loop."""
    if max(m * l, l * n, m * n) > S:
        raise ValueError("shape does not fit one ciphertext")
    tr = _alg1_count(n, l, m, S) < _alg1_count(m, l, n, S)
    mo, no = (n, m) if tr else (m, n)
    region = frozenset(i + j * mo for i in range(mo) for j in range(no))
    eps, omega = [], []
    for k in range(l):
        ce = alg1_eps_diagonals(mo, l, no, k)
        cw = alg1_omega_diagonals(mo, l, no, k)
        eps.append(_terms(ce, region, sorted(ce)))
        omega.append(_terms(cw, region, sorted(cw)))
    if not cloud:
        return Plan(m, l, n, tr, mo, no, 1, l, 1, mo, l, l, eps, omega, [0], method=1)
    cs, ct = sigma_diagonals(mo, l), tau_diagonals(l, no)
    sigma = _terms(cs, frozenset(range(mo * l)), sorted(cs))
    tau = _terms(ct, frozenset(range(l * no)), sorted(ct))
    return Plan(m, l, n, tr, mo, no, 1, l, 1, mo, l, l, eps, omega, [0], method=3, sigma=sigma, tau=tau)


def eps_diagonals(mo: int, lb: int, no: int, M: int, W: int, k: int) -> Dict[int, set]:
    """Nonzero diagonals of eps^k_{M x no} on the packed left operand, as
    {rotation z: output slots}.  Output (i, j) reads source column c = j + k,
    or j + k - lb past the packed width W, i.e. slot i + c*M: a left rotation
    by (c - j)*M.  Row block h = i // mo holds partial product (k + h*mo) mod
    lb (Theorem 5); it is kept only when h*mo + k < lb, so that every partial
    product is accumulated exactly once (the redundant copies of Algorithm 2
    are dropped)."""
    cand: Dict[int, set] = {}
    for i in range(M):
        if (i // mo) * mo + k >= lb:
            continue
        for j in range(no):
            c = j + k if j + k < W else j + k - lb
            cand.setdefault((c - j) * M, set()).add(i + j * M)
    return cand


def omega_diagonals(lb: int, no: int, M: int, k: int) -> Dict[int, set]:
    """Nonzero diagonals of omega^k_{M x no}: output (i, j) reads source row
    r = i + k, or i + k - lb past row M: a left rotation by r - i."""
    cand: Dict[int, set] = {}
    for i in range(M):
        for j in range(no):
            r = i + k if i + k < M else i + k - lb
            cand.setdefault(r - i, set()).add(i + j * M)
    return cand


def _terms(cand: Dict[int, set], region: frozenset, order: Sequence[int]):
    """Diagonal list in a fixed order; a lone diagonal covering the whole
    output region needs no mask (None)."""
    out = []
    for z in order:
        if z in cand and cand[z]:
            out.append((z, frozenset(cand[z])))
    assert sum(len(s) for _, s in out) == sum(len(s) for s in cand.values())
    if len(out) == 1 and out[0][1] == region:
        out = [(out[0][0], None)]
    return out


# ---------------------------------------------------------------------------
# client side: packing and unpacking
# ---------------------------------------------------------------------------

def oriented_operands(pl: Plan, A: np.ndarray, B: np.ndarray):
    A = np.asarray(A, dtype=np.int64)
    B = np.asarray(B, dtype=np.int64)
    if pl.transposed:
        return B.T.copy(), A.T.copy()
    return A, B


def pack_left(pl: Plan, X: np.ndarray, block: int, t: int, S: int) -> List[int]:
    """Algorithm 1: x[i + c*mo] = X[i][(i + c) mod l], sigma(X) column-major.
    Algorithm 2: x[i + c*M] = Xb[i mod mo][(i + c) mod lb] for i < M, c < W: the
    client-side eps^0_{M x W}(sigma(Xbar)) of Algorithm 2, with Xbar the d
    stacked copies of the block Xb, flattened column-major."""
    if pl.method == 1:
        x = [0] * S
        for i in range(pl.mo):
            for c in range(pl.l):
                x[i + c * pl.mo] = int(X[i][(i + c) % pl.l]) % t
        return x
    if pl.method == 3:   # X itself, column-major; sigma is applied in the cloud
        x = [0] * S
        for i in range(pl.mo):
            for c in range(pl.l):
                x[i + c * pl.mo] = int(X[i][c]) % t
        return x
    Xb = np.zeros((pl.mo, pl.lb), dtype=np.int64)
    lo = block * pl.lb
    hi = min(pl.l, lo + pl.lb)
    Xb[:, : hi - lo] = X[:, lo:hi]
    x = [0] * S
    for i in range(pl.M):
        for c in range(pl.W):
            x[i + c * pl.M] = int(Xb[i % pl.mo][(i + c) % pl.lb]) % t
    return x


def pack_right(pl: Plan, Y: np.ndarray, block: int, t: int, S: int) -> List[int]:
    """Algorithm 1: y[r + j*l] = Y[(r + j) mod l][j], tau(Y) column-major.
    Algorithm 2: y[r + j*M] = Yb[(r + j) mod lb][j] for r < M, j < no: the
    client-side omega^0_{M x no}(tau(Yb)), flattened column-major."""
    if pl.method == 1:
        y = [0] * S
        for r in range(pl.l):
            for j in range(pl.no):
                y[r + j * pl.l] = int(Y[(r + j) % pl.l][j]) % t
        return y
    if pl.method == 3:   # Y itself, column-major; tau is applied in the cloud
        y = [0] * S
        for r in range(pl.l):
            for j in range(pl.no):
                y[r + j * pl.l] = int(Y[r][j]) % t
        return y
    Yb = np.zeros((pl.lb, pl.no), dtype=np.int64)
    lo = block * pl.lb
    hi = min(pl.l, lo + pl.lb)
    Yb[: hi - lo, :] = Y[lo:hi, :]
    y = [0] * S
    for r in range(pl.M):
        for j in range(pl.no):
            y[r + j * pl.M] = int(Yb[(r + j) % pl.lb][j]) % t
    return y


def unpack(pl: Plan, slots: Sequence[int]) -> np.ndarray:
    """C[i][j] sits at slot i + j*M, or at j + i*M when the problem was transposed."""
    C = np.zeros((pl.m, pl.n), dtype=np.int64)
    for i in range(pl.m):
        for j in range(pl.n):
            s = (j + i * pl.M) if pl.transposed else (i + j * pl.M)
            C[i, j] = int(slots[s])
    return C


# ---------------------------------------------------------------------------
# cleartext twin: the same plan run on slot vectors mod t
# ---------------------------------------------------------------------------

def _rot_clear(v: Sequence[int], z: int) -> List[int]:
    S = len(v)
    return [v[(s + z) % S] for s in range(S)]


def _rot_sum_clear(v, terms, t):
    S = len(v)
    out = [0] * S
    for z, mask in terms:
        r = _rot_clear(v, z)
        for s in range(S):
            if mask is None or s in mask:
                out[s] = (out[s] + r[s]) % t
    return out


def hegmm_cleartext(pl: Plan, A, B, t: int, S: int) -> np.ndarray:
    """Run the plan on unencrypted slot vectors: the packing/plan check that
    needs no encryption."""
    X, Y = oriented_operands(pl, A, B)
    acc = [0] * S
    for b in range(pl.nb):
        x = pack_left(pl, X, b, t, S)
        y = pack_right(pl, Y, b, t, S)
        if pl.method == 3:
            x = _rot_sum_clear(x, pl.sigma, t)
            y = _rot_sum_clear(y, pl.tau, t)
        for k in range(pl.K):
            e = _rot_sum_clear(x, pl.eps[k], t)
            f = _rot_sum_clear(y, pl.omega[k], t)
            acc = [(acc[s] + e[s] * f[s]) % t for s in range(S)]
    acc = _rot_sum_clear(acc, [(z, None) for z in pl.fold], t)
    return unpack(pl, acc)


# ---------------------------------------------------------------------------
# encrypted run
# ---------------------------------------------------------------------------

class MaskCache:
    def __init__(self, P: Params):
        self.P = P
        self.cache: Dict[frozenset, bgv.Mask] = {}

    def get(self, slots: frozenset) -> bgv.Mask:
        m = self.cache.get(slots)
        if m is None:
            v = [0] * self.P.S
            for s in slots:
                v[s] = 1
            m = bgv.Mask(self.P, v)
            self.cache[slots] = m
        return m


def galois_elements(P: Params, shapes: Sequence[Tuple[int, int, int]], method: int = 2,
                    min_blocks: int = 1) -> List[int]:
    gs = set()
    for (m, l, n) in shapes:
        pl = plan(m, l, n, P.S, method, min_blocks)
        for z in pl.rotations(P.S):
            gs.add(P.galois(z))
    return sorted(gs)


def encrypt_operand(ks: bgv.KeySet, pl: Plan, role: int, A, B, nonce: int) -> List[bgv.Ct]:
    """Client preprocessing (Algorithm 2): pack and encrypt one operand, one
    ciphertext per inner block.  role 0 = left (A side), 1 = right (B side)."""
    P = ks.P
    X, Y = oriented_operands(pl, A, B)
    out = []
    for b in range(pl.nb):
        v = pack_left(pl, X, b, P.t, P.S) if role == 0 else pack_right(pl, Y, b, P.t, P.S)
        out.append(bgv.encrypt_slots(ks, v, role=role, block=b, nonce=nonce))
    return out


def hegmm(ks: bgv.KeySet, pl: Plan, ctX: List[bgv.Ct], ctY: List[bgv.Ct],
          masks: Optional[MaskCache] = None, eager: bool = False, ks_order: int = 0) -> bgv.Ct:
    """Cloud side of Algorithm 2:  Acc = sum_{blocks, k < K} eps^k(ctX) x omega^k(ctY),
    one relinearisation, then the fold sum_h Rot(R, h*mo) that gathers the d
    row blocks (the extraction of Theorem 5's partial products).

    eager=True takes each product of the loop as a full HE-Mult (tensor, then
    relinearisation, the HE-Mult of Section II-A) and sums the relinearised
    two-component ciphertexts; the default relinearises the three-component
    sum once.  Both decrypt to the same matrix; their bits differ (the key
    switch lifts and rounds each input on its own).

    ks_order selects how every linear transform (eps^k, omega^k, sigma, tau,
    the fold) is composed:
      0  rot_sum: the masked key-switching sums of a transform are divided by
         P once (deferred division);
      1  lin_transform: the paper's primitive order of Eq. (lintrans), one
         complete HE-Rot per diagonal (its own division by P), then HE-CMult
         by the mask, then HE-Add.
    Both decrypt to the same matrix; their bits differ."""
    P = ks.P
    masks = masks or MaskCache(P)
    if ks_order not in (0, 1):
        raise ValueError("ks_order must be 0 or 1")
    transform = bgv.lin_transform if ks_order == 1 else bgv.rot_sum

    def terms(tms):
        return [(z, None if s is None else masks.get(s)) for z, s in tms]

    if pl.method == 3:   # sigma and tau of Algorithm 1 on the ciphertexts (Theorems 1 and 2)
        ctX = [transform(P, ks, ctX[0], terms(pl.sigma))]
        ctY = [transform(P, ks, ctY[0], terms(pl.tau))]
    acc = None
    for b in range(pl.nb):
        for k in range(pl.K):
            e = transform(P, ks, ctX[b], terms(pl.eps[k]))
            f = transform(P, ks, ctY[b], terms(pl.omega[k]))
            prod = bgv.he_mult(P, ks, e, f) if eager else bgv.tensor(P, e, f)
            acc = prod if acc is None else bgv.he_add(P, acc, prod)
    R = acc if eager else bgv.relinearize(P, ks, acc)
    if pl.d == 1:
        return R
    return transform(P, ks, R, [(z, None) for z in pl.fold])


def decrypt_result(ks: bgv.KeySet, pl: Plan, ct: bgv.Ct) -> np.ndarray:
    return unpack(pl, bgv.decrypt_slots(ks, ct))


def export_d7(ct: bgv.Ct) -> np.ndarray:
    """Canonical serialisation: coefficient form, components then limbs, u64."""
    return np.concatenate([np.ascontiguousarray(c, dtype=np.uint64).reshape(-1) for c in ct])
