"""Pins for the oracle's HEGMM-En planner, packing and encrypted loop.

Against the paper: the worked examples printed in its figure captions and
text (tests/golden/paper_examples.json), the element-wise identity of
Section III-A written out from the operator definitions, Theorem 5's
coverage.  Against the mathematics: brute-force integer matrix products
(decrypt(HEGMM(Enc A, Enc B)) == A.B mod t)."""
import json
import os
import random

import numpy as np
import pytest

import workloads
from oracle import bgv, hegmm as H
from oracle.ring import Params

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


# ---------------------------------------------------------------------------
# Section III-A written out from the operator definitions (Eqs. sigma..omega)
# ---------------------------------------------------------------------------

def sigma(A):
    m, l = len(A), len(A[0])
    return [[A[i][(i + j) % l] for j in range(l)] for i in range(m)]


def tau(B):
    l, n = len(B), len(B[0])
    return [[B[(i + j) % l][j] for j in range(n)] for i in range(l)]


def eps(A, k, m, n):
    l = len(A[0])
    return [[A[i][(j + k) % l] for j in range(n)] for i in range(m)]


def omega(B, k, m, n):
    l = len(B)
    return [[B[(i + k) % l][j] for j in range(n)] for i in range(m)]


@pytest.mark.parametrize("shape", [(5, 3, 4), (2, 5, 7), (5, 4, 2), (1, 1, 1), (7, 1, 3), (3, 8, 3)])
def test_elementwise_identity(shape):
    m, l, n = shape
    rng = random.Random(sum(shape))
    A = [[rng.randrange(-9, 10) for _ in range(l)] for _ in range(m)]
    B = [[rng.randrange(-9, 10) for _ in range(n)] for _ in range(l)]
    sA, tB = sigma(A), tau(B)
    C = [[0] * n for _ in range(m)]
    for k in range(l):
        e, w = eps(sA, k, m, n), omega(tB, k, m, n)
        for i in range(m):
            for j in range(n):
                C[i][j] += e[i][j] * w[i][j]
    want = [[sum(A[i][k] * B[k][j] for k in range(l)) for j in range(n)] for i in range(m)]
    assert C == want


# ---------------------------------------------------------------------------
# worked examples printed in the paper
# ---------------------------------------------------------------------------

def test_figure_eps_example():
    g = GOLDEN["eps1_5x3"]
    d = H.eps_diagonals(g["M"], g["lb"], g["no"], g["M"], g["W"], g["k"])
    assert {str(z): sorted(s) for z, s in d.items()} == g["diagonals"]


def test_figure_omega_example():
    g = GOLDEN["omega1_3x5"]
    d = H.omega_diagonals(g["lb"], g["no"], g["M"], g["k"])
    assert {str(z): len(s) for z, s in d.items()} == g["diagonal_sizes"]


def _partials(pl, k):
    """Partial products (k + h*mo) mod lb held by the row blocks kept at iteration k."""
    kept = set()
    for z, s in pl.eps[k]:
        slots = range(pl.M * pl.no) if s is None else s
        for x in slots:
            kept.add((x % pl.M) // pl.mo)
    return sorted((k + h * pl.mo) % pl.lb for h in kept)


def test_duplicate_a_example():
    g = GOLDEN["dupA_2x5x7"]
    pl = H.plan(g["m"], g["l"], g["n"], 4096)
    assert not pl.transposed and pl.d == g["d"] and pl.K == 2
    assert _partials(pl, 0) == sorted(g["partials_k0"])
    all_k1 = [(1 + h * pl.mo) % pl.lb for h in range(pl.d)]
    assert all_k1 == g["partials_k1_all"]
    assert _partials(pl, 1) == sorted(g["partials_k1_kept"])


def test_duplicate_b_example():
    g = GOLDEN["dupB_5x4x2"]
    pl = H.plan(g["m"], g["l"], g["n"], 4096)
    assert pl.transposed and pl.d == g["d"] and pl.K == 2
    for k, want in g["partials"].items():
        assert _partials(pl, int(k)) == want


def test_iteration_count_example():
    g = GOLDEN["alg1_5x3x4"]
    pl = H.plan(g["m"], g["l"], g["n"], 4096)
    assert pl.K == g["iterations"]


@pytest.mark.parametrize("shape", [(2, 5, 7), (3, 10, 4), (4, 9, 9), (6, 6, 6), (9, 4, 3), (5, 13, 2)])
def test_theorem5_each_partial_once(shape):
    m, l, n = shape
    pl = H.plan(m, l, n, 4096)
    seen = []
    for k in range(pl.K):
        seen += _partials(pl, k)
    assert sorted(seen) == list(range(pl.lb))
    assert pl.K == min(m, l, n) or pl.K == min(pl.mo, pl.lb)


# ---------------------------------------------------------------------------
# the plan on cleartext slot vectors vs brute-force matrix products
# ---------------------------------------------------------------------------

def test_cleartext_twin_random_shapes():
    rng = np.random.default_rng(11)
    for (m, l, n) in workloads.random_shapes(rng, 150, 1, 12):
        A = rng.integers(-8, 9, size=(m, l))
        B = rng.integers(-8, 9, size=(l, n))
        pl = H.plan(m, l, n, 256)
        assert (H.hegmm_cleartext(pl, A, B, 12289, 256) == workloads.plain_matmul_mod(A, B, 12289)).all(), (m, l, n)
        # at most two diagonals per transform, and <= 2 rotations each
        assert all(len(t) <= 2 for t in pl.eps + pl.omega)


def test_cleartext_twin_blocked_shapes():
    rng = np.random.default_rng(12)
    count = 0
    for (m, l, n) in workloads.random_shapes(rng, 300, 2, 30):
        try:
            pl = H.plan(m, l, n, 64)
        except ValueError:
            assert m * n > 64
            continue
        if pl.nb == 1:
            continue
        count += 1
        A = rng.integers(-8, 9, size=(m, l))
        B = rng.integers(-8, 9, size=(l, n))
        assert (H.hegmm_cleartext(pl, A, B, 12289, 64) == workloads.plain_matmul_mod(A, B, 12289)).all(), (m, l, n)
        if count > 40:
            break
    assert count > 10


def test_forced_blocking_plans():
    """Section IV-D's blockwise product forced on shapes that fit whole: the
    large configuration splits its inner dimension 96 into two blocks of 48;
    blocks never exceed l; the blocked plan is still exact on cleartext."""
    large = H.plan(128, 96, 128, 16384, min_blocks=2)
    assert (large.nb, large.lb, large.M, large.W) == (2, 48, 128, 128)
    assert H.plan(4, 3, 5, 512, min_blocks=9).nb == 3          # capped at l
    assert H.plan(64, 32, 48, 4096, min_blocks=1).nb == 1
    with pytest.raises(ValueError):
        H.plan(4, 3, 5, 512, method=1, min_blocks=2)
    rng = np.random.default_rng(13)
    for (m, l, n) in workloads.random_shapes(rng, 60, 2, 12):
        for k in (2, 3):
            pl = H.plan(m, l, n, 256, min_blocks=k)
            assert pl.nb == min(k, l) and pl.lb == -(-l // pl.nb)
            A = rng.integers(-8, 9, size=(m, l))
            B = rng.integers(-8, 9, size=(l, n))
            assert (H.hegmm_cleartext(pl, A, B, 12289, 256) == workloads.plain_matmul_mod(A, B, 12289)).all(), (m, l, n, k)


def test_headline_plan_counts():
    pl = H.plan(64, 32, 48, 4096)
    assert (pl.transposed, pl.d, pl.M, pl.K, pl.W, pl.nb) == (False, 1, 64, 32, 48, 1)
    assert len(pl.rotations(4096)) == 124
    tiny = H.plan(4, 3, 5, 512)
    assert sorted(z if z < 256 else z - 512 for z in tiny.rotations(512)) == [-8, -4, -2, -1, 1, 2, 4, 8]
    large = H.plan(128, 96, 128, 16384)
    assert large.nb == 1 and large.M * large.W == 16384


def test_batched_grid_fit_counts():
    grid = range(8, 65, 8)
    fit = sum(1 for m in grid for l in grid for n in grid if H.plan(m, l, n, 4096).nb == 1)
    assert fit == 468


# ---------------------------------------------------------------------------
# encrypted end to end
# ---------------------------------------------------------------------------

def run_encrypted(P, shapes, seed, min_blocks=1):
    ks = bgv.KeySet(P, seed, H.galois_elements(P, shapes, min_blocks=min_blocks))
    rng = np.random.default_rng(seed)
    masks = H.MaskCache(P)
    for idx, (m, l, n) in enumerate(shapes):
        A = rng.integers(-8, 9, size=(m, l))
        B = rng.integers(-8, 9, size=(l, n))
        pl = H.plan(m, l, n, P.S, min_blocks=min_blocks)
        cx = H.encrypt_operand(ks, pl, 0, A, B, nonce=idx)
        cy = H.encrypt_operand(ks, pl, 1, A, B, nonce=idx)
        C = H.hegmm(ks, pl, cx, cy, masks)
        assert len(C) == 2
        got = H.decrypt_result(ks, pl, C)
        assert (got == workloads.plain_matmul_mod(A, B, P.t)).all(), (m, l, n)


def test_encrypted_small_shapes_alpha1():
    P = Params(128, 12289, 3, 1)
    # d > 1 (fold), transposed, l-min, square, blocked (M*W > 64)
    run_encrypted(P, [(2, 5, 7), (5, 4, 2), (6, 3, 5), (4, 4, 4), (3, 11, 6), (1, 6, 1)], 77)


def test_encrypted_forced_blocks():
    """Forced inner blocks (one accumulator over the block products) decrypt
    to A B mod t."""
    P = Params(128, 12289, 3, 1)
    run_encrypted(P, [(2, 5, 7), (5, 4, 2), (4, 4, 4)], 79, min_blocks=2)


def test_encrypted_small_shapes_alpha2():
    P = Params(128, 12289, 4, 2)
    run_encrypted(P, [(3, 7, 5), (7, 5, 3), (2, 9, 4)], 78)


def _noise_and_bits(P, shapes, seed, min_blocks=1):
    """Both transform orders on the same encrypted operands: per shape the
    decryptions, the noise of each result and whether their bits differ."""
    ks = bgv.KeySet(P, seed, H.galois_elements(P, shapes, min_blocks=min_blocks))
    rng = np.random.default_rng(seed)
    masks = H.MaskCache(P)
    out = []
    for idx, (m, l, n) in enumerate(shapes):
        A = rng.integers(-8, 9, size=(m, l))
        B = rng.integers(-8, 9, size=(l, n))
        pl = H.plan(m, l, n, P.S, min_blocks=min_blocks)
        cx = H.encrypt_operand(ks, pl, 0, A, B, nonce=idx)
        cy = H.encrypt_operand(ks, pl, 1, A, B, nonce=idx)
        want = workloads.plain_matmul_mod(A, B, P.t)
        res = {}
        for order in (0, 1):
            C = H.hegmm(ks, pl, cx, cy, masks, ks_order=order)
            assert (H.decrypt_result(ks, pl, C) == want).all(), ((m, l, n), order)
            res[order] = (C, bgv.noise_bits(ks, C, bgv.decrypt_poly(ks, C)))
        differ = any((x != y).any() for x, y in zip(res[0][0], res[1][0]))
        out.append(((m, l, n), pl, res[0][1], res[1][1], differ))
    return out


@pytest.mark.parametrize("alpha", [1, 2])
def test_paper_order_decrypts_like_deferred(alpha):
    """HEGMM-En with every transform in the paper's primitive order (one
    HE-Rot, HE-CMult, HE-Add per diagonal) and with the deferred division by P
    decrypt to the same A.B mod t on fold (2x5x7), transposed (5x4x2),
    inner-blocked (3x11x6) and square shapes, at alpha = 1 and alpha = 2.
    Their noise agrees within a quarter bit (neither order is noisier; the
    mask times the input noise dominates both), and products whose transforms
    carry masks give different bits."""
    P = Params(128, 12289, 3 + alpha - 1, alpha)
    shapes = [(2, 5, 7), (5, 4, 2), (3, 11, 6), (4, 4, 4)]
    cases = set()
    for (m, l, n), pl, nb_def, nb_pap, differ in _noise_and_bits(P, shapes, 80 + alpha):
        shape = (m, l, n)
        assert abs(nb_def - nb_pap) <= 0.25, (shape, nb_def, nb_pap)
        assert nb_pap < np.log2(float(P.Q)) - 2, shape
        masked = any(s is not None for t in pl.eps + pl.omega for _, s in t)
        assert differ == masked, shape
        cases |= {c for c, on in (("fold", pl.d > 1), ("transposed", pl.transposed), ("blocked", pl.nb > 1),
                                  ("square", m == l == n)) if on}
    assert cases == {"fold", "transposed", "blocked", "square"}


def test_tiny_config_end_to_end():
    cfg = workloads.TINY
    P = Params(cfg.N, cfg.t, cfg.L, cfg.alpha)
    A, B = workloads.tiny_operands()
    pl = H.plan(4, 3, 5, P.S)
    ks = bgv.KeySet(P, cfg.seed, H.galois_elements(P, [(4, 3, 5)]))
    cx = H.encrypt_operand(ks, pl, 0, A, B, nonce=1)
    cy = H.encrypt_operand(ks, pl, 1, A, B, nonce=1)
    C = H.hegmm(ks, pl, cx, cy)
    assert (H.decrypt_result(ks, pl, C) == workloads.plain_matmul_mod(A, B, P.t)).all()
    mu = bgv.decrypt_poly(ks, C)
    assert bgv.noise_bits(ks, C, mu) < np.log2(float(P.Q)) - 2


# ---------------------------------------------------------------------------
# Algorithm 1 (HEGMM) variant
# ---------------------------------------------------------------------------

def test_alg1_figure_diagonals():
    """The eps^1 / omega^1 examples of the transform figure (Section III-B):
    Algorithm 1 flattens column-major without duplication, so its diagonals
    are exactly the captioned ones."""
    g = GOLDEN["eps1_5x3"]
    got = {z: sorted(s) for z, s in H.alg1_eps_diagonals(5, 3, 3, 1).items()}
    assert got == {int(z): v for z, v in g["diagonals"].items()}
    g = GOLDEN["omega1_3x5"]
    got = {z: len(s) for z, s in H.alg1_omega_diagonals(3, 3, 5, 1).items()}
    assert got == {int(z): v for z, v in g["diagonal_sizes"].items()}


def test_alg1_iterations_and_eps_bound():
    """l iterations (the mm-example figure: 5x3 times 3x4 takes 3), and at
    most ceil(n/l) + 1 diagonals per eps^k in column-major (corrected
    Theorem 3)."""
    g = GOLDEN["alg1_5x3x4"]
    assert H.plan(g["m"], g["l"], g["n"], 4096, method=1).K == g["iterations"]
    for m in range(1, 9):
        for l in range(1, 9):
            for n in range(1, 9):
                for k in range(l):
                    assert len(H.alg1_eps_diagonals(m, l, n, k)) <= -(-n // l) + 1


@pytest.mark.parametrize("shape", [(5, 3, 3), (3, 3, 5), (4, 3, 5), (2, 5, 7), (7, 3, 2), (6, 4, 9), (1, 6, 1), (9, 1, 4)])
def test_alg1_cleartext_twin(shape):
    m, l, n = shape
    rng = np.random.default_rng(m * 100 + l * 10 + n)
    A = rng.integers(-8, 9, size=(m, l))
    B = rng.integers(-8, 9, size=(l, n))
    pl = H.plan(m, l, n, 512, method=1)
    assert pl.method == 1 and pl.d == 1 and pl.nb == 1 and pl.K == l
    assert np.array_equal(H.hegmm_cleartext(pl, A, B, 12289, 512), workloads.plain_matmul_mod(A, B, 12289))


def test_alg1_needs_more_rotations_than_en():
    """The point of Algorithm 2: on the headline shape HEGMM-En needs far
    fewer key-switched rotations than Algorithm 1."""
    en = H.plan(64, 32, 48, 4096)
    a1 = H.plan(64, 32, 48, 4096, method=1)
    count = lambda pl: sum(1 for ts in pl.eps + pl.omega for z, _ in ts if z % 4096)
    assert count(a1) > 2 * count(en)


def test_alg1_encrypted_small():
    c = workloads.TINY
    P = Params(c.N, c.t, c.L, c.alpha)
    shapes = [(4, 3, 5), (3, 5, 2)]
    ks = bgv.KeySet(P, c.seed, H.galois_elements(P, shapes, method=1))
    rng = np.random.default_rng(8)
    for (m, l, n) in shapes:
        A = rng.integers(-8, 9, size=(m, l))
        B = rng.integers(-8, 9, size=(l, n))
        pl = H.plan(m, l, n, P.S, method=1)
        ox = H.encrypt_operand(ks, pl, 0, A, B, 3)
        oy = H.encrypt_operand(ks, pl, 1, A, B, 3)
        C = H.decrypt_result(ks, pl, H.hegmm(ks, pl, ox, oy))
        assert np.array_equal(C, workloads.plain_matmul_mod(A, B, c.t)), (m, l, n)


# ---------------------------------------------------------------------------
# eager relinearisation (HE-Mult per loop product)
# ---------------------------------------------------------------------------

def test_eager_relin_decrypts():
    """Each loop product relinearised on its own (HE-Mult as in Section II-A):
    the sum still decrypts to A B mod t on every plan shape (fold, transposed,
    blocked, forced blocks), with noise well inside the modulus."""
    P = Params(128, 12289, 3, 1)
    shapes = [(2, 5, 7), (5, 4, 2), (4, 4, 4), (3, 11, 6)]
    ks = bgv.KeySet(P, 81, H.galois_elements(P, shapes) + H.galois_elements(P, shapes[:2], min_blocks=2))
    rng = np.random.default_rng(81)
    masks = H.MaskCache(P)
    for idx, (m, l, n) in enumerate(shapes + [(2, 5, 7)]):
        mb = 2 if idx == len(shapes) else 1
        A = rng.integers(-8, 9, size=(m, l))
        B = rng.integers(-8, 9, size=(l, n))
        pl = H.plan(m, l, n, P.S, min_blocks=mb)
        cx = H.encrypt_operand(ks, pl, 0, A, B, nonce=idx)
        cy = H.encrypt_operand(ks, pl, 1, A, B, nonce=idx)
        C = H.hegmm(ks, pl, cx, cy, masks, eager=True)
        assert len(C) == 2
        assert (H.decrypt_result(ks, pl, C) == workloads.plain_matmul_mod(A, B, P.t)).all(), (m, l, n)
        mu = bgv.decrypt_poly(ks, C)
        assert bgv.noise_bits(ks, C, mu) < np.log2(float(P.Q)) - 2
        if pl.nb * pl.K > 1:
            # more than one product: relinearising each on its own changes the bits
            lazy = H.hegmm(ks, pl, cx, cy, masks)
            assert not np.array_equal(H.export_d7(C), H.export_d7(lazy)), (m, l, n)


def test_eager_relin_single_product_equals_lazy():
    """With one loop product (K = 1, one block) eager and lazy
    relinearisation are the same computation: bit-identical ciphertexts."""
    P = Params(128, 12289, 3, 1)
    shapes = [(1, 4, 3), (5, 1, 2)]
    ks = bgv.KeySet(P, 82, H.galois_elements(P, shapes))
    rng = np.random.default_rng(82)
    for idx, (m, l, n) in enumerate(shapes):
        pl = H.plan(m, l, n, P.S)
        assert pl.nb * pl.K == 1
        A = rng.integers(-8, 9, size=(m, l))
        B = rng.integers(-8, 9, size=(l, n))
        cx = H.encrypt_operand(ks, pl, 0, A, B, nonce=idx)
        cy = H.encrypt_operand(ks, pl, 1, A, B, nonce=idx)
        e = H.hegmm(ks, pl, cx, cy, eager=True)
        z = H.hegmm(ks, pl, cx, cy)
        assert np.array_equal(H.export_d7(e), H.export_d7(z))
        assert (H.decrypt_result(ks, pl, e) == workloads.plain_matmul_mod(A, B, P.t)).all()


# ---------------------------------------------------------------------------
# Algorithm 1 with sigma and tau evaluated in the cloud (method 3)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(5, 3, 4), (3, 5, 2), (4, 4, 4), (1, 6, 2), (7, 2, 3), (2, 7, 6)])
def test_cloud_sigma_tau_diagonals(shape):
    """The sigma / tau rotation sums reproduce the Section III-A definitions
    sigma(X)[i][j] = X[i][(i+j) mod l], tau(Y)[i][j] = Y[(i+j) mod l][j] on the
    column-major slot vectors, with 2 min(mo, l) - 1 and 2 min(no, l) - 1
    diagonals (Theorems 1 and 2; both bounds are met here).  Theorem 1's
    claim that row-major flattening has the same count is checked from the
    definition directly."""
    m, l, n = shape
    S, t = 64, 257
    pl = H.plan(m, l, n, S, method=3)
    assert pl.method == 3
    rng = np.random.default_rng(sum(shape))
    X = rng.integers(0, t, size=(pl.mo, l))
    Y = rng.integers(0, t, size=(l, pl.no))
    x = [0] * S
    x[: pl.mo * l] = [int(v) for v in X.flatten(order="F")]
    y = [0] * S
    y[: l * pl.no] = [int(v) for v in Y.flatten(order="F")]
    sx = np.array([[X[i, (i + j) % l] for j in range(l)] for i in range(pl.mo)])
    ty = np.array([[Y[(i + j) % l, j] for j in range(pl.no)] for i in range(l)])
    want_x = [0] * S
    want_x[: pl.mo * l] = [int(v) for v in sx.flatten(order="F")]
    want_y = [0] * S
    want_y[: l * pl.no] = [int(v) for v in ty.flatten(order="F")]
    assert H._rot_sum_clear(x, pl.sigma, t) == want_x
    assert H._rot_sum_clear(y, pl.tau, t) == want_y
    assert len(pl.sigma) == 2 * min(pl.mo, l) - 1
    assert len(pl.tau) == 2 * min(pl.no, l) - 1
    # row-major: slot i*l + j of sigma(X) reads slot i*l + (i+j) mod l
    rm = {i * l + (i + j) % l - (i * l + j) for i in range(pl.mo) for j in range(l)}
    assert len(rm) <= 2 * min(pl.mo, l) - 1


def test_cloud_sigma_tau_encrypted():
    """Method 3 end to end: the sigma / tau passes on the encrypted plain
    packing decrypt to the client-side sigma / tau packing of Algorithm 1,
    and the product decrypts to A B mod t."""
    P = Params(128, 12289, 3, 1)
    shapes = [(4, 3, 5), (3, 5, 2), (2, 4, 6)]
    ks = bgv.KeySet(P, 83, H.galois_elements(P, shapes, method=3))
    rng = np.random.default_rng(83)
    masks = H.MaskCache(P)
    for idx, (m, l, n) in enumerate(shapes):
        A = rng.integers(-8, 9, size=(m, l))
        B = rng.integers(-8, 9, size=(l, n))
        pl = H.plan(m, l, n, P.S, method=3)
        p1 = H.plan(m, l, n, P.S, method=1)
        assert (pl.transposed, pl.eps, pl.omega) == (p1.transposed, p1.eps, p1.omega)
        cx = H.encrypt_operand(ks, pl, 0, A, B, nonce=idx)
        cy = H.encrypt_operand(ks, pl, 1, A, B, nonce=idx)
        X, Y = H.oriented_operands(pl, A, B)
        sx = bgv.rot_sum(P, ks, cx[0], [(z, None if s is None else masks.get(s)) for z, s in pl.sigma])
        ty = bgv.rot_sum(P, ks, cy[0], [(z, None if s is None else masks.get(s)) for z, s in pl.tau])
        assert bgv.decrypt_slots(ks, sx) == H.pack_left(p1, X, 0, P.t, P.S)
        assert bgv.decrypt_slots(ks, ty) == H.pack_right(p1, Y, 0, P.t, P.S)
        C = H.hegmm(ks, pl, cx, cy, masks)
        assert (H.decrypt_result(ks, pl, C) == workloads.plain_matmul_mod(A, B, P.t)).all(), (m, l, n)
        assert (H.hegmm_cleartext(pl, A, B, P.t, P.S) == workloads.plain_matmul_mod(A, B, P.t)).all()
