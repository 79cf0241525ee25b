/*
 * Plain CPU reference arithmetic for BGV over RNS (test infrastructure).
 *
 * This file is part of the ORACLE: a slow, obviously correct model that the
 * GPU library is checked against.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code with the
 * GPU library.
 *
 * Every modular product is a 128-bit product followed by a `%` reduction; no
 * Barrett, Montgomery or Shoup tricks.  Each polynomial is stored as rows of
 * N unsigned 64-bit residues (one row per prime, coefficient or evaluation
 * form as each function states).  Loops over independent rows carry an
 * OpenMP pragma; that changes no result.
 *
 * What is computed follows the paper's HE primitive set (Section II-A:
 * HE-Add, HE-Mult, HE-CMult, HE-Rot) over the ring Z_q[X]/(X^N+1) of
 * Section IV-A, realised as BGV with hybrid key switching.  The paper is
 * silent on the key-switching method; the conventions used here are the
 * ones written down in the design notes (special-modulus key switching with
 * digits of alpha primes, centered lifts everywhere, t-corrected division
 * by P).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t u64;
typedef int64_t i64;
typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ */
/* scalar modular arithmetic                                            */
/* ------------------------------------------------------------------ */

static u64 mulmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }
static u64 addmod(u64 a, u64 b, u64 q) { u64 s = a + b; return s >= q ? s - q : s; }
static u64 submod(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + (q - b); }

/* x (any signed 64-bit value) reduced into [0, q) */
static u64 reduce_signed(i64 x, u64 q) {
    i64 r = x % (i64)q;
    if (r < 0) r += (i64)q;
    return (u64)r;
}

/* centered representative of x in [0,q): value in (-q/2, q/2] (q odd, so no tie) */
static i64 centered(u64 x, u64 q) { return x > q / 2 ? (i64)x - (i64)q : (i64)x; }

u64 or_powmod(u64 a, u64 e, u64 q) {
    u64 r = 1 % q;
    a %= q;
    while (e) {
        if (e & 1) r = mulmod(r, a, q);
        a = mulmod(a, a, q);
        e >>= 1;
    }
    return r;
}

/* inverse modulo a prime q by Fermat's little theorem */
u64 or_invmod(u64 a, u64 q) { return or_powmod(a, q - 2, q); }

/* ------------------------------------------------------------------ */
/* negacyclic number-theoretic transform                                */
/* ------------------------------------------------------------------ */

/* In-place cyclic DFT of length N over Z_q with root w (w^N = 1):
 * A[i] = sum_j a[j] w^(i j).  Textbook iterative radix-2: bit-reversal
 * permutation followed by log2(N) stages of Cooley-Tukey butterflies. */
static void cyclic_dft(u64 *a, int N, u64 q, u64 w) {
    for (int i = 1, j = 0; i < N; ++i) {
        int bit = N >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { u64 t = a[i]; a[i] = a[j]; a[j] = t; }
    }
    for (int len = 2; len <= N; len <<= 1) {
        u64 wl = or_powmod(w, (u64)(N / len), q);
        for (int s = 0; s < N; s += len) {
            u64 wk = 1;
            for (int k = 0; k < len / 2; ++k) {
                u64 u = a[s + k];
                u64 v = mulmod(a[s + k + len / 2], wk, q);
                a[s + k] = addmod(u, v, q);
                a[s + k + len / 2] = submod(u, v, q);
                wk = mulmod(wk, wl, q);
            }
        }
    }
}

/* Forward negacyclic transform, natural order:
 *   out[i] = a(psi^(2i+1)) = sum_j a[j] psi^((2i+1) j)  (mod q)
 * where psi is a primitive 2N-th root of unity.  Computed as the cyclic DFT
 * (root psi^2) of the twisted vector a[j] psi^j. */
void or_ntt(u64 *a, int N, u64 q, u64 psi) {
    u64 pj = 1;
    for (int j = 0; j < N; ++j) { a[j] = mulmod(a[j], pj, q); pj = mulmod(pj, psi, q); }
    cyclic_dft(a, N, q, mulmod(psi, psi, q));
}

/* Inverse of or_ntt: coefficients from the natural-order evaluations. */
void or_intt(u64 *a, int N, u64 q, u64 psi) {
    u64 psi_inv = or_invmod(psi, q);
    cyclic_dft(a, N, q, mulmod(psi_inv, psi_inv, q));
    u64 n_inv = or_invmod((u64)N % q, q);
    u64 pj = n_inv;
    for (int j = 0; j < N; ++j) { a[j] = mulmod(a[j], pj, q); pj = mulmod(pj, psi_inv, q); }
}

void or_ntt_rows(u64 *a, int rows, int N, const u64 *q, const u64 *psi) {
#pragma omp parallel for schedule(dynamic)
    for (int r = 0; r < rows; ++r) or_ntt(a + (size_t)r * N, N, q[r], psi[r]);
}

void or_intt_rows(u64 *a, int rows, int N, const u64 *q, const u64 *psi) {
#pragma omp parallel for schedule(dynamic)
    for (int r = 0; r < rows; ++r) or_intt(a + (size_t)r * N, N, q[r], psi[r]);
}

/* Schoolbook product in Z_q[X]/(X^N+1): X^N = -1 folds the upper half back
 * with a sign flip.  O(N^2); used only to pin the transform. */
void or_negacyclic_schoolbook(u64 *out, const u64 *a, const u64 *b, int N, u64 q) {
    for (int k = 0; k < N; ++k) out[k] = 0;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            u64 p = mulmod(a[i], b[j], q);
            int k = i + j;
            if (k < N) out[k] = addmod(out[k], p, q);
            else out[k - N] = submod(out[k - N], p, q);
        }
}

/* ------------------------------------------------------------------ */
/* row-wise pointwise operations (rows x N, row r uses prime q[r])      */
/* ------------------------------------------------------------------ */

void or_mul_rows(u64 *out, const u64 *a, const u64 *b, int rows, int N, const u64 *q) {
#pragma omp parallel for
    for (int r = 0; r < rows; ++r)
        for (int i = 0; i < N; ++i) {
            size_t x = (size_t)r * N + i;
            out[x] = mulmod(a[x], b[x], q[r]);
        }
}

void or_add_rows(u64 *out, const u64 *a, const u64 *b, int rows, int N, const u64 *q) {
#pragma omp parallel for
    for (int r = 0; r < rows; ++r)
        for (int i = 0; i < N; ++i) {
            size_t x = (size_t)r * N + i;
            out[x] = addmod(a[x], b[x], q[r]);
        }
}

void or_sub_rows(u64 *out, const u64 *a, const u64 *b, int rows, int N, const u64 *q) {
#pragma omp parallel for
    for (int r = 0; r < rows; ++r)
        for (int i = 0; i < N; ++i) {
            size_t x = (size_t)r * N + i;
            out[x] = submod(a[x], b[x], q[r]);
        }
}

/* out[r][i] = a[r][i] * c[r] mod q[r] */
void or_scale_rows(u64 *out, const u64 *a, const u64 *c, int rows, int N, const u64 *q) {
#pragma omp parallel for
    for (int r = 0; r < rows; ++r)
        for (int i = 0; i < N; ++i) {
            size_t x = (size_t)r * N + i;
            out[x] = mulmod(a[x], c[r] % q[r], q[r]);
        }
}

/* out[r][i] = x[i] mod q[r] for a signed integer polynomial x */
void or_reduce_signed_rows(u64 *out, const i64 *x, int rows, int N, const u64 *q) {
    for (int r = 0; r < rows; ++r)
        for (int i = 0; i < N; ++i) out[(size_t)r * N + i] = reduce_signed(x[i], q[r]);
}

/* Galois automorphism X -> X^g (g odd) in coefficient form: coefficient j
 * moves to position j*g mod 2N, negated when that position is >= N. */
void or_automorph_rows(u64 *out, const u64 *a, int rows, int N, const u64 *q, u64 g) {
    u64 twoN = 2 * (u64)N;
    for (int r = 0; r < rows; ++r) {
        const u64 *ar = a + (size_t)r * N;
        u64 *o = out + (size_t)r * N;
        for (int j = 0; j < N; ++j) {
            u64 pos = ((u64)j * g) % twoN;
            if (pos < (u64)N) o[pos] = ar[j];
            else o[pos - N] = ar[j] == 0 ? 0 : q[r] - ar[j];
        }
    }
}

/* ------------------------------------------------------------------ */
/* pseudo-random streams (SplitMix64, Steele-Lea-Flood 2014)            */
/* ------------------------------------------------------------------ */

#define GOLDEN_GAMMA 0x9E3779B97F4A7C15ULL

u64 or_mix64(u64 z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* starting state of the stream owned by object (tag, idx) under a master seed */
u64 or_stream_seed(u64 master, u64 tag, u64 idx) {
    return or_mix64(or_mix64(or_mix64(master) ^ tag) ^ idx);
}

/* k-th output (k = 0, 1, ...) of the SplitMix64 sequence started at s0 */
static u64 draw(u64 s0, u64 k) { return or_mix64(s0 + (k + 1) * GOLDEN_GAMMA); }

/* high 64 bits of r * m: a value in [0, m) */
static u64 scale_draw(u64 r, u64 m) { return (u64)(((u128)r * m) >> 64); }

/* rows x N uniform residues; row r coefficient i uses draw first + r*N + i */
void or_sample_uniform(u64 *out, u64 s0, u64 first, int rows, int N, const u64 *q) {
    for (int r = 0; r < rows; ++r)
        for (int i = 0; i < N; ++i) {
            u64 k = first + (u64)r * N + i;
            out[(size_t)r * N + i] = scale_draw(draw(s0, k), q[r]);
        }
}

/* ternary coefficients: 0 -> 0, 1 -> +1, 2 -> -1 */
void or_sample_ternary(i64 *out, u64 s0, u64 first, int N) {
    for (int i = 0; i < N; ++i) {
        u64 v = scale_draw(draw(s0, first + i), 3);
        out[i] = v == 0 ? 0 : (v == 1 ? 1 : -1);
    }
}

/* discrete Gaussian by cumulative table: x = lo + #{k : cdt[k] <= r} */
void or_sample_cdt(i64 *out, u64 s0, u64 first, int N, const u64 *cdt, int ncdt, i64 lo) {
    for (int i = 0; i < N; ++i) {
        u64 r = draw(s0, first + i);
        i64 c = 0;
        for (int k = 0; k < ncdt; ++k) c += (cdt[k] <= r);
        out[i] = lo + c;
    }
}

/* ------------------------------------------------------------------ */
/* key switching: digit lift (ModUp) and t-corrected division (ModDown) */
/* ------------------------------------------------------------------ */

/* ext[] lists the extended basis: ext[0..L-1] = q_0..q_{L-1},
 * ext[L..L+alpha-1] = p_0..p_{alpha-1}. */

/* Lift one digit of c to the whole extended basis (coefficient form).
 * c: L rows over q (coefficient form).  The digit holds primes q_d0..q_{d1-1}
 * with product D.  For a prime r outside the digit:
 *   y_r = sum_{i in digit} ctilde_i * (D/q_i)  mod r,
 *   ctilde_i = centered( c_i * (D/q_i)^{-1} mod q_i ).
 * For a prime inside the digit y_r = c_r. */
void or_modup_digit(u64 *y, const u64 *c, int N, int L, int alpha, const u64 *ext, int d0, int d1) {
    int nd = d1 - d0;
    u64 inv_hat[8];
    for (int a = 0; a < nd; ++a) {
        u64 qi = ext[d0 + a];
        u64 hat = 1;
        for (int b = 0; b < nd; ++b)
            if (b != a) hat = mulmod(hat, ext[d0 + b] % qi, qi);
        inv_hat[a] = or_invmod(hat, qi);
    }
#pragma omp parallel for
    for (int r = 0; r < L + alpha; ++r) {
        u64 pr = ext[r];
        u64 *yr = y + (size_t)r * N;
        if (r >= d0 && r < d1) {
            memcpy(yr, c + (size_t)r * N, sizeof(u64) * N);
            continue;
        }
        u64 hat_mod_r[8];
        for (int a = 0; a < nd; ++a) {
            u64 h = 1;
            for (int b = 0; b < nd; ++b)
                if (b != a) h = mulmod(h, ext[d0 + b] % pr, pr);
            hat_mod_r[a] = h;
        }
        for (int i = 0; i < N; ++i) {
            u64 acc = 0;
            for (int a = 0; a < nd; ++a) {
                u64 qi = ext[d0 + a];
                i64 ct = centered(mulmod(c[(size_t)(d0 + a) * N + i], inv_hat[a], qi), qi);
                acc = addmod(acc, mulmod(reduce_signed(ct, pr), hat_mod_r[a], pr), pr);
            }
            yr[i] = acc;
        }
    }
}

/* Divide by P with a correction that keeps the plaintext (mod t) intact.
 * u: (L+alpha) rows, coefficient form, extended basis.  out: L rows over q.
 *   r_k     = centered( u_{p_k} * t^{-1} * (P/p_k)^{-1} mod p_k )
 *   delta_i = t * sum_k r_k * (P/p_k)  mod q_i
 *   out_i   = (u_{q_i} - delta_i) * P^{-1}  mod q_i
 * delta is congruent to u modulo P and to 0 modulo t, so (u - delta)/P is
 * an exact integer division that leaves the message mod t unchanged. */
void or_moddown(u64 *out, const u64 *u, int N, int L, int alpha, const u64 *ext, u64 t) {
    const u64 *p = ext + L;
    u64 coef[8];  /* t^{-1} * (P/p_k)^{-1} mod p_k */
    for (int k = 0; k < alpha; ++k) {
        u64 hat = 1;
        for (int b = 0; b < alpha; ++b)
            if (b != k) hat = mulmod(hat, p[b] % p[k], p[k]);
        coef[k] = mulmod(or_invmod(t % p[k], p[k]), or_invmod(hat, p[k]), p[k]);
    }
    i64 *rk = (i64 *)malloc(sizeof(i64) * (size_t)alpha * N);
    for (int k = 0; k < alpha; ++k)
        for (int i = 0; i < N; ++i)
            rk[(size_t)k * N + i] = centered(mulmod(u[(size_t)(L + k) * N + i], coef[k], p[k]), p[k]);
#pragma omp parallel for
    for (int r = 0; r < L; ++r) {
        u64 qi = ext[r];
        u64 hat_q[8];
        for (int k = 0; k < alpha; ++k) {
            u64 h = 1;
            for (int b = 0; b < alpha; ++b)
                if (b != k) h = mulmod(h, p[b] % qi, qi);
            hat_q[k] = h;
        }
        u64 Pq = 1;
        for (int k = 0; k < alpha; ++k) Pq = mulmod(Pq, p[k] % qi, qi);
        u64 Pinv = or_invmod(Pq, qi);
        u64 tq = t % qi;
        for (int i = 0; i < N; ++i) {
            u64 s = 0;
            for (int k = 0; k < alpha; ++k)
                s = addmod(s, mulmod(reduce_signed(rk[(size_t)k * N + i], qi), hat_q[k], qi), qi);
            u64 delta = mulmod(tq, s, qi);
            out[(size_t)r * N + i] = mulmod(submod(u[(size_t)r * N + i], delta, qi), Pinv, qi);
        }
    }
    free(rk);
}
