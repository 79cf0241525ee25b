// Host-side number theory for parameter set-up: modular arithmetic on
// 64-bit words through 128-bit products, primality, roots of unity.
#pragma once
#include <cstdint>
#include <vector>

namespace hg {

using u64 = uint64_t;
using i64 = int64_t;
using u128 = unsigned __int128;

inline u64 hmul(u64 a, u64 b, u64 m) { return (u64)((u128)a * b % m); }
inline u64 hadd(u64 a, u64 b, u64 m) { u64 s = a + b; return s >= m ? s - m : s; }
inline u64 hsub(u64 a, u64 b, u64 m) { return a >= b ? a - b : a + (m - b); }

inline u64 hpow(u64 b, u64 e, u64 m) {
    u64 r = 1 % m;
    b %= m;
    while (e) {
        if (e & 1) r = hmul(r, b, m);
        b = hmul(b, b, m);
        e >>= 1;
    }
    return r;
}

// inverse modulo a prime (Fermat)
inline u64 hinv(u64 a, u64 p) { return hpow(a % p, p - 2, p); }

// signed value reduced into [0, m)
inline u64 hred(i64 x, u64 m) {
    i64 r = x % (i64)m;
    return (u64)(r < 0 ? r + (i64)m : r);
}

// Miller-Rabin, deterministic below 2^64 with the first twelve prime bases.
inline bool is_prime_u64(u64 n) {
    if (n < 2) return false;
    static const u64 bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (u64 p : bases)
        if (n % p == 0) return n == p;
    u64 d = n - 1;
    int s = 0;
    while ((d & 1) == 0) { d >>= 1; ++s; }
    for (u64 a : bases) {
        u64 x = hpow(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int i = 1; i < s; ++i) {
            x = hmul(x, x, n);
            if (x == n - 1) { comp = false; break; }
        }
        if (comp) return false;
    }
    return true;
}

// The first `count` primes below 2^bits with p = 1 (mod 2N), descending.
inline std::vector<u64> find_ntt_primes(u64 N, int count, int bits = 50) {
    std::vector<u64> out;
    u64 step = 2 * N;
    u64 k = ((1ULL << bits) - 2) / step;
    while ((int)out.size() < count && k > 0) {
        u64 p = k * step + 1;
        if (p < (1ULL << bits) && is_prime_u64(p)) out.push_back(p);
        --k;
    }
    return out;
}

// A primitive 2N-th root of unity mod prime p (p = 1 mod 2N): x^((p-1)/2N)
// for the first x >= 2 whose power has order exactly 2N.  The root fixes the
// evaluation points, and key a_j values are drawn directly as evaluations,
// so this rule is part of the key convention.
inline u64 find_psi(u64 p, u64 N) {
    u64 e = (p - 1) / (2 * N);
    for (u64 x = 2;; ++x) {
        u64 w = hpow(x, e, p);
        if (hpow(w, N, p) == p - 1) return w;
    }
}

// zeta_t: the smallest x in [2, t) with x^N = -1 (mod t).  This choice fixes
// which evaluation point each slot is, so it is part of the encoding.
inline u64 smallest_neg_root(u64 t, u64 N) {
    for (u64 x = 2; x < t; ++x)
        if (hpow(x, N, t) == t - 1) return x;
    return 0;
}

inline uint32_t bitrev(uint32_t x, int bits) {
    uint32_t r = 0;
    for (int i = 0; i < bits; ++i) { r = (r << 1) | (x & 1); x >>= 1; }
    return r;
}

inline i64 centered_of(u64 x, u64 m) { return x > m / 2 ? (i64)x - (i64)m : (i64)x; }

}  // namespace hg
