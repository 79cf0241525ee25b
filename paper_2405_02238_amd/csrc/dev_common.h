// Device helpers shared by the kernel files.
#pragma once
#include <hip/hip_runtime.h>

namespace hg {

__device__ __forceinline__ int brev_bits(int x, int bits) {
    return (int)(__brev((unsigned)x) >> (32 - bits));
}

// Evaluation-form automorphism X -> X^g: position p holds the value at
// psi^(2 brv(p) + 1).  The permuted polynomial's value there is the source
// value at psi^((2 brv(p) + 1) g): natural index ((2i+1) g mod 2N - 1) / 2.
// For 64 consecutive positions (an aligned block) the sources form a
// permutation of another aligned block of 64, so the gather stays coalesced.
__device__ __forceinline__ int perm_index(int p, int g, int logN) {
    int i = brev_bits(p, logN);
    int twoN = 2 << logN;
    int e = (int)(((long long)(2 * i + 1) * g) & (twoN - 1));
    return brev_bits((e - 1) >> 1, logN);
}

// Every buffer the kernels touch lives in global memory, but a pointer read
// out of a descriptor table is generic to the compiler, which then emits
// flat loads and stores; those also count as scalar-memory operations, so a
// wait for a scalar load (the next table entry) stalls until they land.
// Accessing through these casts gives plain global instructions.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *gld(const T *p) {
    return (const __attribute__((address_space(1))) T *)p;
}
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gst(T *p) {
    return (__attribute__((address_space(1))) T *)p;
}

}  // namespace hg
