// Exact modular arithmetic on the FP64 vector units of gfx950.
//
// Residues modulo a prime q < 2^50 are held as doubles that are exact
// integers.  Every value kept in memory lies in (-q, q) (a signed, not
// necessarily reduced, representative); the canonical forms are produced
// only where the integer itself matters (centered lifts, export).
//
// Product a*b mod q with |a|, |b| < q (so |ab| < 2^100):
//   h = fl(a*b), l = fma(a, b, -h)   -- h + l = ab exactly (FMA error term)
//   e = rint(h * (1/q))              -- quotient estimate, off by < 1
//   r = fma(-e, q, h) + l            -- both steps exact: |h - e q| < 2^51
// gives |r| < 0.875 q.  This is the floating-point modular multiplication of
// van der Hoeven, Lecerf and Quintin ("Modular SIMD arithmetic in
// Mathemagix", 2016), chosen over 64-bit integer Shoup/Barrett products
// because the integer multipliers of gfx950 are measured slower (FP64 FMA is
// full rate on this chip).  Every step is an IEEE correctly rounded
// operation, so the results are deterministic and exact.
#pragma once
#include <hip/hip_runtime.h>

namespace hg {

struct ModQ {
    double q, qi;  // prime and fl(1/q)
};

// |a|, |b| < q  ->  r = a*b (mod q), |r| < 0.875 q
__device__ __forceinline__ double mulm(double a, double b, double q, double qi) {
    double h = a * b;
    double l = __fma_rn(a, b, -h);
    double e = rint(h * qi);
    double r = __fma_rn(-e, q, h);
    return r + l;
}

// any integer-valued |x| < 2^53  ->  x (mod q) with |r| <= q/2 + 1 (x * fl(1/q)
// is then within 2^-49 of x/q, so the estimated quotient is off by at most
// one at a near-tie, and the fused remainder is an exact small integer)
__device__ __forceinline__ double redm(double x, double q, double qi) {
    return __fma_rn(-rint(x * qi), q, x);
}

// |x| < q  ->  the centered representative in (-q/2, q/2), exactly.
// (x/q is at least 1/(2q) away from any half-integer because q is odd, and
// the rounding error of x * fl(1/q) is below 2^-52 for |x| < q.)
__device__ __forceinline__ double centerm(double x, double q, double qi) {
    return __fma_rn(-rint(x * qi), q, x);
}

// |x| < q  ->  the canonical representative in [0, q)
__device__ __forceinline__ double canonm(double x, double q) {
    return x < 0.0 ? x + q : x;
}

__device__ __forceinline__ double addm(double a, double b, double q, double qi) {
    return redm(a + b, q, qi);
}

__device__ __forceinline__ double subm(double a, double b, double q, double qi) {
    return redm(a - b, q, qi);
}

}  // namespace hg
