// Negacyclic number-theoretic transforms on gfx950.
//
// Forward: Cooley-Tukey with the 2N-th root psi merged into the twiddles
// (Poeppelmann-Oder-Gueneysu 2015; Longa-Naehrig 2016), natural order in,
// bit-reversed order out: position p holds a(psi^(2 brv(p) + 1)).
// Inverse: Gentleman-Sande with psi^-1 twiddles, bit-reversed in, natural
// out, scaled by N^-1.
//
// One workgroup owns one row (one prime of one polynomial); the row lives in
// LDS, padded by one double every 16 so that the strided accesses of the late
// rounds hit distinct banks.  Each round runs three or four radix-2 stages in
// registers on the 8 or 16 elements of one group per thread; the first round
// of a forward transform takes its inputs from registers and its last round
// writes the outputs, and the inverse mirrors this, so an 8192-point row
// (13 stages: 3+3+3+3+1) makes three full LDS round trips.  Reductions are
// lazy: forward stages reduce every fourth stage (values below 7q in between),
// inverse rows of up to 2^14 points reduce their sums every second stage;
// all within the exact range of the FP64 arithmetic (below 2^53).
//
// The load and store steps fuse the neighbouring work of key switching:
// LOAD_MODUP lifts one digit of a coefficient-form polynomial to the prime of
// the row (ModUp), LOAD_DELTA forms the correction delta of the division by P
// from the centered r_k rows, STORE_MDR turns an inverse-transformed special
// prime row into the exact centered r_k.
#include <hip/hip_ext.h>

#include <stdexcept>

#include "arith.h"
#include "dev_common.h"
#include "kernels.h"

namespace hg {

namespace {

constexpr int NTT_THREADS_MAX = 1024;
constexpr int SPLIT_ELEMS = 4096;            // elements per workgroup in the split transform
constexpr int SPLIT_THREADS = SPLIT_ELEMS / 16;

__device__ __forceinline__ int lds_ix(int i) { return i + (i >> 4); }

// LDS index of element base + b * TS.  When TS is a multiple of 16 the
// padding term splits, so every element sits at a constant offset from the
// first (immediate offsets in the LDS instructions instead of index math).
template <int TS>
__device__ __forceinline__ int lds_ix_step(int base, int b) {
    if constexpr (TS % 16 == 0) return lds_ix(base) + b * (TS + TS / 16);
    else return lds_ix(base + b * TS);
}

// log2 of the radix of the whole-row transforms: each thread owns 2^RK
// elements per round, so a row uses N / 2^RK threads.  Radix 8 for 4096- and
// 8192-point rows (more waves per row to hide FP64 and LDS latency), radix
// 16 otherwise.
__host__ __device__ constexpr int rk_of(int logn) { return (logn == 12 || logn == 13) ? 3 : 4; }

// Minimum waves per SIMD asked of the compiler for the row kernels: with
// 1024-thread rows (8192 points) two rows fit a CU (LDS 2 x 70 KB) when each
// thread keeps to 64 VGPRs, i.e. 8 waves per SIMD; other sizes keep the
// default.
__host__ __device__ constexpr int waves_of(int logn, int rk) { return logn == 13 ? (rk == 3 ? 8 : 4) : 1; }

// ---- whole rows with the size known at compile time ----
// Round R of a 2^LOGN-point forward transform covers stages [S0, S0 + K).
// Each thread owns a group of 2^K elements; all twiddles of the round are
// loaded into registers before the butterflies, so one memory latency is paid
// per round, and whether a stage reduces is decided at compile time.
template <int LOGN, int S0, int K>
__device__ __forceinline__ void fwd_round_c(double *sh, const double *__restrict__ tw, double q, double qi) {
    constexpr int N = 1 << LOGN;
    constexpr int LTS = LOGN - S0 - K;
    constexpr int TS = 1 << LTS;
    constexpr int NG = N >> K;
    for (int grp = threadIdx.x; grp < NG; grp += blockDim.x) {
        const int low = grp & (TS - 1);
        const int blk = grp >> LTS;
        const int base = (blk << (LTS + K)) + low;
        double w[(1 << K) - 1];
#pragma unroll
        for (int u = 0; u < K; ++u)
#pragma unroll
            for (int c = 0; c < (1 << u); ++c) w[(1 << u) - 1 + c] = tw[(1 << (S0 + u)) + (blk << u) + c];
        double x[1 << K];
#pragma unroll
        for (int b = 0; b < (1 << K); ++b) x[b] = sh[lds_ix_step<TS>(base, b)];
#pragma unroll
        for (int u = 0; u < K; ++u) {
            constexpr int dummy = 0;
            (void)dummy;
            const bool red = ((S0 + u) & 1) || (S0 + u == LOGN - 1);
            const int half = 1 << (K - 1 - u);
#pragma unroll
            for (int b = 0; b < (1 << K); ++b) {
                if (b & half) continue;
                const double t = mulm(x[b + half], w[(1 << u) - 1 + (b >> (K - u))], q, qi);
                const double X = x[b];
                if (red) {
                    x[b] = redm(X + t, q, qi);
                    x[b + half] = redm(X - t, q, qi);
                } else {
                    x[b] = X + t;
                    x[b + half] = X - t;
                }
            }
        }
#pragma unroll
        for (int b = 0; b < (1 << K); ++b) sh[lds_ix_step<TS>(base, b)] = x[b];
    }
}

template <int LOGN, int S0>
__device__ __forceinline__ void fwd_rows_c(double *sh, const double *tw, double q, double qi) {
    if constexpr (S0 < LOGN) {
        constexpr int RK = rk_of(LOGN);
        constexpr int K = (LOGN - S0) < RK ? (LOGN - S0) : RK;
        fwd_round_c<LOGN, S0, K>(sh, tw, q, qi);
        __syncthreads();
        fwd_rows_c<LOGN, S0 + K>(sh, tw, q, qi);
    }
}

template <int LOGN, int LTS, int K>
__device__ __forceinline__ void inv_round_c(double *sh, const double *__restrict__ tw, double q, double qi) {
    constexpr int N = 1 << LOGN;
    constexpr int TS = 1 << LTS;
    constexpr int NG = N >> K;
    for (int grp = threadIdx.x; grp < NG; grp += blockDim.x) {
        const int low = grp & (TS - 1);
        const int blk = grp >> LTS;
        const int base = (blk << (LTS + K)) + low;
        // stage u needs 2^(K-u-1) twiddles; offsets within w: 0, 2^(K-1), ...
        double w[(1 << K) - 1];
        int wo = 0;
#pragma unroll
        for (int u = 0; u < K; ++u) {
#pragma unroll
            for (int c = 0; c < (1 << (K - u - 1)); ++c)
                w[wo + c] = tw[(N >> (LTS + u + 1)) + (blk << (K - u - 1)) + c];
            wo += 1 << (K - u - 1);
        }
        double x[1 << K];
#pragma unroll
        for (int b = 0; b < (1 << K); ++b) x[b] = sh[lds_ix_step<TS>(base, b)];
        wo = 0;
#pragma unroll
        for (int u = 0; u < K; ++u) {
            const int d = 1 << u;
#pragma unroll
            for (int b = 0; b < (1 << K); ++b) {
                if (b & d) continue;
                const double X = x[b], Y = x[b + d];
                x[b] = redm(X + Y, q, qi);
                x[b + d] = mulm(X - Y, w[wo + (b >> (u + 1))], q, qi);
            }
            wo += 1 << (K - u - 1);
        }
#pragma unroll
        for (int b = 0; b < (1 << K); ++b) sh[lds_ix_step<TS>(base, b)] = x[b];
    }
}

template <int LOGN, int LTS>
__device__ __forceinline__ void inv_rows_c(double *sh, const double *tw, double q, double qi) {
    if constexpr (LTS < LOGN) {
        constexpr int RK = rk_of(LOGN);
        constexpr int K = (LOGN - LTS) < RK ? (LOGN - LTS) : RK;
        inv_round_c<LOGN, LTS, K>(sh, tw, q, qi);
        __syncthreads();
        inv_rows_c<LOGN, LTS + K>(sh, tw, q, qi);
    }
}

// ---- whole rows with both ends in registers (2^10 .. 2^14 points) ----
// A row of N = 2^LOGN points runs on NT = N / 2^RK threads.  The forward
// transform takes the 2^RK elements t + b NT of thread t straight from the
// caller (global memory, or the registers an inverse transform left) into
// its first round, and hands the outputs of its last round to a store
// functor; the inverse transform reads global memory in its first round and
// leaves the outputs of its last round, again elements t + b NT, in
// registers.  Against staging the row through LDS at both ends, this saves
// two LDS round trips and two barriers per transform, and a chain inverse ->
// elementwise step -> forward keeps the row in registers in between.
// Forward rounds: RK, ..., RK, KT; inverse rounds: KT, RK, ..., RK
// (KT = the remainder of LOGN over RK, or RK).
template <int LOGN, int RK_ = rk_of(LOGN)>
struct Rows {
    static constexpr int N = 1 << LOGN;
    static constexpr int RK = RK_;
    static constexpr int NT = N >> RK;                          // threads per row
    static constexpr int KT = LOGN % RK == 0 ? RK : LOGN % RK;  // stages of the short round
    static constexpr int SL = LOGN - KT;                        // forward: first stage of the short round
    static constexpr int GPT = 1 << (RK - KT);                  // short-round groups per thread
};

template <int LOGN>
__host__ __device__ constexpr bool direct_rows() { return LOGN >= 10 && LOGN <= 14; }

// Twiddles of forward stages [S0, S0 + K) for group blk.
template <int S0, int K>
__device__ __forceinline__ void fwd_tw(double *w, const double *__restrict__ tw, int blk) {
#pragma unroll
    for (int u = 0; u < K; ++u)
#pragma unroll
        for (int c = 0; c < (1 << u); ++c) w[(1 << u) - 1 + c] = tw[(1 << (S0 + u)) + (blk << u) + c];
}

// Forward stages [S0, S0 + K) on the 2^K elements of one group.  Stages
// 3, 7, 11, ... and the last one reduce.  A twiddle product (twiddles are
// centered, below q/2) is below 1.5q even with both roundings of the
// quotient estimate off, so from inputs below 2q the values stay below 7q
// before each reduction: under 2^53 (q < 2^50), where redm and mulm are
// exact, and the residues do not depend on the reduction schedule.
template <int LOGN, int S0, int K>
__device__ __forceinline__ void fwd_bfly(double *x, const double *w, double q, double qi) {
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const bool red = ((S0 + u) % 4 == 3) || (S0 + u == LOGN - 1);
        const int half = 1 << (K - 1 - u);
#pragma unroll
        for (int b = 0; b < (1 << K); ++b) {
            if (b & half) continue;
            const double t = mulm(x[b + half], w[(1 << u) - 1 + (b >> (K - u))], q, qi);
            const double X = x[b];
            if (red) {
                x[b] = redm(X + t, q, qi);
                x[b + half] = redm(X - t, q, qi);
            } else {
                x[b] = X + t;
                x[b + half] = X - t;
            }
        }
    }
}

// Twiddles of the inverse round whose first stage has half-size 2^LTS0.
template <int LOGN, int LTS0, int K>
__device__ __forceinline__ void inv_tw(double *w, const double *__restrict__ tw, int blk) {
    constexpr int N = 1 << LOGN;
    int wo = 0;
#pragma unroll
    for (int u = 0; u < K; ++u) {
#pragma unroll
        for (int c = 0; c < (1 << (K - u - 1)); ++c) w[wo + c] = tw[(N >> (LTS0 + u + 1)) + (blk << (K - u - 1)) + c];
        wo += 1 << (K - u - 1);
    }
}

// Inverse stages of half-size 2^LTS0 .. 2^(LTS0 + K - 1) on one group.  The
// sums are reduced on odd stages and the last one, the differences always
// go through a twiddle product.  With the bound on twiddle products above
// and inputs below q (stored rows are reduced), every value of a row of up
// to 2^14 points stays below 7.3q < 2^53; the outputs (last differences)
// are below 2q, and every consumer multiplies them before anything else.
template <int LOGN, int LTS0, int K>
__device__ __forceinline__ void inv_bfly(double *x, const double *w, double q, double qi) {
    int wo = 0;
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const int d = 1 << u;
        const bool red = ((LTS0 + u) & 1) || (LTS0 + u == LOGN - 1);
#pragma unroll
        for (int b = 0; b < (1 << K); ++b) {
            if (b & d) continue;
            const double X = x[b], Y = x[b + d];
            x[b] = red ? redm(X + Y, q, qi) : X + Y;
            x[b + d] = mulm(X - Y, w[wo + (b >> (u + 1))], q, qi);
        }
        wo += 1 << (K - u - 1);
    }
}

// Full forward rounds from stage S0 up to the short round, one group per
// thread, the next round's twiddles loaded while this one computes.
// SG = 1, hb = h: the transform is half h of a 2^(LOGN + 1)-point row whose
// first stage has been applied, i.e. its local stage s is the row's stage
// s + 1 and its group blk at local stage s is the row's group (h << s) + blk.
template <int LOGN, int RKX, int S0, int SG = 0>
__device__ __forceinline__ void fwd_mid(double *sh, const double *__restrict__ tw, double q, double qi, int t,
                                        const double *wcur, int hb = 0) {
    using R = Rows<LOGN, RKX>;
    if constexpr (S0 < R::SL) {
        constexpr int K = R::RK, LTS = LOGN - S0 - K, TS = 1 << LTS;
        constexpr int S1 = S0 + K;
        const int low = t & (TS - 1);
        const int base = ((t >> LTS) << (LTS + K)) + low;
        double x[1 << K];
#pragma unroll
        for (int b = 0; b < (1 << K); ++b) x[b] = sh[lds_ix_step<TS>(base, b)];
        double wnext[(1 << K) - 1];
        if constexpr (S1 < R::SL) fwd_tw<S1 + SG, K>(wnext, tw, (hb << S1) + (t >> (LOGN - S1 - K)));
        fwd_bfly<LOGN + SG, S0 + SG, K>(x, wcur, q, qi);
#pragma unroll
        for (int b = 0; b < (1 << K); ++b) sh[lds_ix_step<TS>(base, b)] = x[b];
        __syncthreads();
        fwd_mid<LOGN, RKX, S1, SG>(sh, tw, q, qi, t, wnext, hb);
    }
}

// No value to combine with an output (fwd_row_regs' default `pre`).
struct NoPre {
    __device__ double operator()(int) const { return 0.0; }
};

// Forward transform of a row of which thread t holds elements t + b NT in
// x (|x| < q); st(i, v, u) receives output position i (bit-reversed order)
// with u = pre(i).  Every pre(i) and the last round's twiddles are loaded
// before the first st: a store through a pointer the compiler cannot tell
// apart from theirs would otherwise keep each of those loads behind the
// store before it.  Uses sh as scratch; the caller must not touch sh
// concurrently.  With SG = 1 the row is half hb of a twice longer row after
// that row's first stage (see fwd_mid; st then receives positions within
// the half).
template <int LOGN, int RKX, int SG = 0, class Store, class Pre = NoPre>
__device__ __forceinline__ void fwd_row_regs(double *sh, const double *__restrict__ tw, double q, double qi,
                                             double *x, Store st, int hb = 0, Pre pre = Pre()) {
    using R = Rows<LOGN, RKX>;
    constexpr int K = R::RK, NT = R::NT, KT = R::KT, SL = R::SL;
    const int t = threadIdx.x;
    double w0[(1 << K) - 1], w1[(1 << K) - 1];
    fwd_tw<SG, K>(w0, tw, hb);
    fwd_tw<K + SG, K>(w1, tw, (hb << K) + (t >> (LOGN - 2 * K)));
    fwd_bfly<LOGN + SG, SG, K>(x, w0, q, qi);
#pragma unroll
    for (int b = 0; b < (1 << K); ++b) sh[lds_ix_step<NT>(t, b)] = x[b];
    __syncthreads();
    fwd_mid<LOGN, RKX, K, SG>(sh, tw, q, qi, t, w1, hb);
    double wl[R::GPT][(1 << KT) - 1], u[R::GPT][1 << KT];
#pragma unroll
    for (int g = 0; g < R::GPT; ++g) {
        const int grp = t + g * NT;
        fwd_tw<SL + SG, KT>(wl[g], tw, (hb << SL) + grp);
#pragma unroll
        for (int b = 0; b < (1 << KT); ++b) u[g][b] = pre((grp << KT) + b);
    }
#pragma unroll
    for (int g = 0; g < R::GPT; ++g) {
        const int grp = t + g * NT;
        double y[1 << KT];
#pragma unroll
        for (int b = 0; b < (1 << KT); ++b) y[b] = sh[lds_ix((grp << KT) + b)];
        fwd_bfly<LOGN + SG, SL + SG, KT>(y, wl[g], q, qi);
#pragma unroll
        for (int b = 0; b < (1 << KT); ++b) st((grp << KT) + b, y[b], u[g][b]);
    }
}

// The forward transform of the register-held row x (thread t: elements
// t + b NT, NT = 2^(LOGN - RKX)) restricted to output half h: the row's first
// stage pairs elements b and b + 2^(RKX-1) of each thread, so the thread
// keeps X + w Y (h = 0) or X - w Y (h = 1) and the rest is an independent
// 2^(LOGN-1)-point transform at radix 2^(RKX-1) on the same NT threads; st
// and pre receive the half's output positions h 2^(LOGN-1) + i.  Two
// workgroups, one per half, finish a row in about the time of one half.
template <int LOGN, int RKX, class Store, class Pre = NoPre>
__device__ __forceinline__ void fwd_row_regs_half(double *sh, const double *__restrict__ tw, double q, double qi,
                                                  double *x, Store st, int h, Pre pre = Pre()) {
    constexpr int HALF = 1 << (RKX - 1);
    const double w = tw[1];
    double z[HALF];
#pragma unroll
    for (int b = 0; b < HALF; ++b) {
        const double t = mulm(x[b + HALF], w, q, qi);
        z[b] = h ? x[b] - t : x[b] + t;
    }
    fwd_row_regs<LOGN - 1, RKX - 1, 1>(
        sh, tw, q, qi, z, [&](int i, double v, double u) { st((h << (LOGN - 1)) + i, v, u); }, h,
        [&](int i) { return pre((h << (LOGN - 1)) + i); });
}

// Full inverse rounds from half-size 2^LTS0 up to the last round.
// SG = 1, hb = h: the transform is the first LOGN stages of a 2^(LOGN + 1)-
// point inverse on input half h (which they do not mix with the other
// half); its group blk of 2^(LTS + K) elements is the row's group
// (h << (LOGN - LTS - K)) + blk.
template <int LOGN, int RKX, int LTS0, int SG = 0>
__device__ __forceinline__ void inv_mid(double *sh, const double *__restrict__ tw, double q, double qi, int t,
                                        const double *wcur, int hb = 0) {
    using R = Rows<LOGN, RKX>;
    if constexpr (LTS0 < LOGN - R::RK) {
        constexpr int K = R::RK, TS = 1 << LTS0, L1 = LTS0 + K;
        const int low = t & (TS - 1);
        const int base = ((t >> LTS0) << (LTS0 + K)) + low;
        double x[1 << K];
#pragma unroll
        for (int b = 0; b < (1 << K); ++b) x[b] = sh[lds_ix_step<TS>(base, b)];
        double wnext[(1 << K) - 1];
        if constexpr (L1 < LOGN - K)
            inv_tw<LOGN + SG, L1, K>(wnext, tw, (hb << (LOGN - L1 - K)) + (t >> L1));
        inv_bfly<LOGN + SG, LTS0, K>(x, wcur, q, qi);
#pragma unroll
        for (int b = 0; b < (1 << K); ++b) sh[lds_ix_step<TS>(base, b)] = x[b];
        __syncthreads();
        inv_mid<LOGN, RKX, L1, SG>(sh, tw, q, qi, t, wnext, hb);
    }
}

// Inverse transform (without the N^-1 scaling) of the row read through
// ld(i) (bit-reversed order); on return thread t holds output positions
// t + b NT in x, |x| < 2q.  sh is scratch.  With SG = 1 the row is input
// half hb of a twice longer row and the transform stops before that row's
// last stage (see inv_mid).
template <int LOGN, int RKX, int SG = 0, class Load>
__device__ __forceinline__ void inv_row_direct(double *sh, const double *__restrict__ tw, double q, double qi, Load ld,
                                               double *x, int hb = 0) {
    using R = Rows<LOGN, RKX>;
    constexpr int K = R::RK, NT = R::NT, KT = R::KT;
    const int t = threadIdx.x;
#pragma unroll
    for (int g = 0; g < R::GPT; ++g) {
        const int grp = t + g * NT;
        double w[(1 << KT) - 1], y[1 << KT];
        inv_tw<LOGN + SG, 0, KT>(w, tw, (hb << (LOGN - KT)) + grp);
#pragma unroll
        for (int b = 0; b < (1 << KT); ++b) y[b] = ld((grp << KT) + b);
        inv_bfly<LOGN + SG, 0, KT>(y, w, q, qi);
#pragma unroll
        for (int b = 0; b < (1 << KT); ++b) sh[lds_ix((grp << KT) + b)] = y[b];
    }
    double w1[(1 << K) - 1];
    if constexpr (KT < LOGN - K) inv_tw<LOGN + SG, KT, K>(w1, tw, (hb << (LOGN - KT - K)) + (t >> KT));
    __syncthreads();
    inv_mid<LOGN, RKX, KT, SG>(sh, tw, q, qi, t, w1, hb);
    double w[(1 << K) - 1];
    inv_tw<LOGN + SG, LOGN - K, K>(w, tw, hb);
#pragma unroll
    for (int b = 0; b < (1 << K); ++b) x[b] = sh[lds_ix_step<NT>(t, b)];
    inv_bfly<LOGN + SG, LOGN - K, K>(x, w, q, qi);
}

// K forward stages [s0, s0 + K) of nsub independent 2^ls-point transforms
// stored one after another in LDS.  Sub-transform sb takes its stage-s
// twiddles from tw[C * 2^s + local], C = cb + sb * cs (C = 1 for a whole row
// or for the columns of a split row; 2^a + block for the blocks of a split
// row).  Stage s is global stage sg0 + s; global stages 3, 7, 11, ..., the
// last global stage, and (force_last) the last local stage reduce their
// outputs (the bound of the row transforms: below 7q in between).
template <int K>
__device__ __forceinline__ void fwd_round(double *sh, const double *__restrict__ tw, int ls, int nsub, int s0,
                                          int cb, int cs, int sg0, int logN, bool force_last, double q, double qi) {
    const int lts = ls - s0 - K;
    const int ts = 1 << lts;
    const int lgps = ls - K;  // log2 groups per sub-transform
    const int ngroups = nsub << lgps;
    for (int grp = threadIdx.x; grp < ngroups; grp += blockDim.x) {
        const int sb = grp >> lgps;
        const int lg = grp & ((1 << lgps) - 1);
        const int low = lg & (ts - 1);
        const int blk = lg >> lts;
        const int base = (sb << ls) + (blk << (lts + K)) + low;
        const int C = cb + sb * cs;
        double x[1 << K];
#pragma unroll
        for (int b = 0; b < (1 << K); ++b) x[b] = sh[lds_ix(base + b * ts)];
#pragma unroll
        for (int u = 0; u < K; ++u) {
            const int s = s0 + u;
            const int sg = sg0 + s;
            const bool red = (sg % 4 == 3) || (sg == logN - 1) || (force_last && s == ls - 1);
            const int half = 1 << (K - 1 - u);
            const double *twu = tw + (C << s) + (blk << u);
#pragma unroll
            for (int b = 0; b < (1 << K); ++b) {
                if (b & half) continue;
                const double w = twu[b >> (K - u)];
                const double t = mulm(x[b + half], w, q, qi);
                const double X = x[b];
                if (red) {
                    x[b] = redm(X + t, q, qi);
                    x[b + half] = redm(X - t, q, qi);
                } else {
                    x[b] = X + t;
                    x[b + half] = X - t;
                }
            }
        }
#pragma unroll
        for (int b = 0; b < (1 << K); ++b) sh[lds_ix(base + b * ts)] = x[b];
    }
}

// K inverse stages of nsub independent 2^ls-point transforms; the first
// stage has half-size 2^lts.  Twiddles tw[C * (2^ls >> (lt + 1)) + local].
template <int K>
__device__ __forceinline__ void inv_round(double *sh, const double *__restrict__ tw, int ls, int nsub, int lts,
                                          int cb, int cs, double q, double qi) {
    const int n = 1 << ls;
    const int ts = 1 << lts;
    const int lgps = ls - K;
    const int ngroups = nsub << lgps;
    for (int grp = threadIdx.x; grp < ngroups; grp += blockDim.x) {
        const int sb = grp >> lgps;
        const int lg = grp & ((1 << lgps) - 1);
        const int low = lg & (ts - 1);
        const int blk = lg >> lts;
        const int base = (sb << ls) + (blk << (lts + K)) + low;
        const int C = cb + sb * cs;
        double x[1 << K];
#pragma unroll
        for (int b = 0; b < (1 << K); ++b) x[b] = sh[lds_ix(base + b * ts)];
#pragma unroll
        for (int u = 0; u < K; ++u) {
            const int d = 1 << u;
            const double *twu = tw + (n >> (lts + u + 1)) * C + (blk << (K - u - 1));
#pragma unroll
            for (int b = 0; b < (1 << K); ++b) {
                if (b & d) continue;
                const double w = twu[b >> (u + 1)];
                const double X = x[b], Y = x[b + d];
                x[b] = redm(X + Y, q, qi);
                x[b + d] = mulm(X - Y, w, q, qi);
            }
        }
#pragma unroll
        for (int b = 0; b < (1 << K); ++b) sh[lds_ix(base + b * ts)] = x[b];
    }
}

// All forward stages [s0, ls) of the sub-transforms, in rounds of four.
__device__ __forceinline__ void fwd_stages(double *sh, const double *tw, int ls, int nsub, int s0, int cb, int cs,
                                           int sg0, int logN, bool force_last, double q, double qi) {
    for (; s0 + 4 <= ls; s0 += 4) {
        fwd_round<4>(sh, tw, ls, nsub, s0, cb, cs, sg0, logN, force_last, q, qi);
        __syncthreads();
    }
    switch (ls - s0) {
        case 3: fwd_round<3>(sh, tw, ls, nsub, s0, cb, cs, sg0, logN, force_last, q, qi); __syncthreads(); break;
        case 2: fwd_round<2>(sh, tw, ls, nsub, s0, cb, cs, sg0, logN, force_last, q, qi); __syncthreads(); break;
        case 1: fwd_round<1>(sh, tw, ls, nsub, s0, cb, cs, sg0, logN, force_last, q, qi); __syncthreads(); break;
        default: break;
    }
}

__device__ __forceinline__ void inv_stages(double *sh, const double *tw, int ls, int nsub, int cb, int cs, double q,
                                           double qi) {
    int lts = 0;
    for (; lts + 4 <= ls; lts += 4) {
        inv_round<4>(sh, tw, ls, nsub, lts, cb, cs, q, qi);
        __syncthreads();
    }
    switch (ls - lts) {
        case 3: inv_round<3>(sh, tw, ls, nsub, lts, cb, cs, q, qi); __syncthreads(); break;
        case 2: inv_round<2>(sh, tw, ls, nsub, lts, cb, cs, q, qi); __syncthreads(); break;
        case 1: inv_round<1>(sh, tw, ls, nsub, lts, cb, cs, q, qi); __syncthreads(); break;
        default: break;
    }
}

// Compile-time forms of the rounds above for the split transforms of a
// known size: shapes, reduction pattern and twiddle offsets are constants and
// each group's twiddles are loaded before its butterflies.
template <int K, int LS, int NSUB, int S0, int SG0, int LOGN, bool FL>
__device__ __forceinline__ void fwd_round_t(double *sh, const double *__restrict__ tw, int cb, int cs, double q,
                                            double qi) {
    constexpr int LTS = LS - S0 - K;
    constexpr int TS = 1 << LTS;
    constexpr int LGPS = LS - K;
    constexpr int NG = NSUB << LGPS;
    for (int grp = threadIdx.x; grp < NG; grp += blockDim.x) {
        const int sb = grp >> LGPS;
        const int lg = grp & ((1 << LGPS) - 1);
        const int low = lg & (TS - 1);
        const int blk = lg >> LTS;
        const int base = (sb << LS) + (blk << (LTS + K)) + low;
        const int C = cb + sb * cs;
        double w[(1 << K) - 1];
#pragma unroll
        for (int u = 0; u < K; ++u)
#pragma unroll
            for (int c = 0; c < (1 << u); ++c) w[(1 << u) - 1 + c] = tw[(C << (S0 + u)) + (blk << u) + c];
        double x[1 << K];
#pragma unroll
        for (int b = 0; b < (1 << K); ++b) x[b] = sh[lds_ix_step<TS>(base, b)];
#pragma unroll
        for (int u = 0; u < K; ++u) {
            constexpr int dummy = 0;
            (void)dummy;
            const int s = S0 + u;
            const int sg = SG0 + s;
            const bool red = (sg % 4 == 3) || (sg == LOGN - 1) || (FL && s == LS - 1);
            const int half = 1 << (K - 1 - u);
#pragma unroll
            for (int b = 0; b < (1 << K); ++b) {
                if (b & half) continue;
                const double t = mulm(x[b + half], w[(1 << u) - 1 + (b >> (K - u))], q, qi);
                const double X = x[b];
                if (red) {
                    x[b] = redm(X + t, q, qi);
                    x[b + half] = redm(X - t, q, qi);
                } else {
                    x[b] = X + t;
                    x[b + half] = X - t;
                }
            }
        }
#pragma unroll
        for (int b = 0; b < (1 << K); ++b) sh[lds_ix_step<TS>(base, b)] = x[b];
    }
}

template <int LS, int NSUB, int S0, int SG0, int LOGN, bool FL>
__device__ __forceinline__ void fwd_stages_t(double *sh, const double *tw, int cb, int cs, double q, double qi) {
    if constexpr (S0 < LS) {
        constexpr int K = (LS - S0) < 4 ? (LS - S0) : 4;
        fwd_round_t<K, LS, NSUB, S0, SG0, LOGN, FL>(sh, tw, cb, cs, q, qi);
        __syncthreads();
        fwd_stages_t<LS, NSUB, S0 + K, SG0, LOGN, FL>(sh, tw, cb, cs, q, qi);
    }
}

// Inverse butterflies of one group of 2^K elements (stages of half-size
// 1, 2, ..., 2^(K-1) within the group), every sum reduced; w holds the
// twiddles stage by stage (2^(K-1), then 2^(K-2), ... of them).
template <int K>
__device__ __forceinline__ void inv_bfly_red(double *x, const double *w, double q, double qi) {
    int wo = 0;
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const int d = 1 << u;
#pragma unroll
        for (int b = 0; b < (1 << K); ++b) {
            if (b & d) continue;
            const double X = x[b], Y = x[b + d];
            x[b] = redm(X + Y, q, qi);
            x[b + d] = mulm(X - Y, w[wo + (b >> (u + 1))], q, qi);
        }
        wo += 1 << (K - u - 1);
    }
}

template <int K, int LS, int NSUB, int LTS>
__device__ __forceinline__ void inv_round_t(double *sh, const double *__restrict__ tw, int cb, int cs, double q,
                                            double qi) {
    constexpr int TS = 1 << LTS;
    constexpr int LGPS = LS - K;
    constexpr int NG = NSUB << LGPS;
    for (int grp = threadIdx.x; grp < NG; grp += blockDim.x) {
        const int sb = grp >> LGPS;
        const int lg = grp & ((1 << LGPS) - 1);
        const int low = lg & (TS - 1);
        const int blk = lg >> LTS;
        const int base = (sb << LS) + (blk << (LTS + K)) + low;
        const int C = cb + sb * cs;
        double w[(1 << K) - 1];
        int wo = 0;
#pragma unroll
        for (int u = 0; u < K; ++u) {
#pragma unroll
            for (int c = 0; c < (1 << (K - u - 1)); ++c)
                w[wo + c] = tw[((1 << LS) >> (LTS + u + 1)) * C + (blk << (K - u - 1)) + c];
            wo += 1 << (K - u - 1);
        }
        double x[1 << K];
#pragma unroll
        for (int b = 0; b < (1 << K); ++b) x[b] = sh[lds_ix_step<TS>(base, b)];
        inv_bfly_red<K>(x, w, q, qi);
#pragma unroll
        for (int b = 0; b < (1 << K); ++b) sh[lds_ix_step<TS>(base, b)] = x[b];
    }
}

template <int LS, int NSUB, int LTS>
__device__ __forceinline__ void inv_stages_t(double *sh, const double *tw, int cb, int cs, double q, double qi) {
    if constexpr (LTS < LS) {
        constexpr int K = (LS - LTS) < 4 ? (LS - LTS) : 4;
        inv_round_t<K, LS, NSUB, LTS>(sh, tw, cb, cs, q, qi);
        __syncthreads();
        inv_stages_t<LS, NSUB, LTS + K>(sh, tw, cb, cs, q, qi);
    }
}

// ---- per-row addressing and the fused load / store steps ----

struct FwdRow {
    int prime;
    double *out;
    const double *in;    // PLAIN: the row; MODUP: the source's L coefficient rows; DELTA: r_k rows
    const double *aux;   // DELTA: the U row
    int d0, d1;          // MODUP: digit primes
};

template <int LOAD>
__device__ __forceinline__ FwdRow fwd_row(const DevTables &T, const NttArgs &a, int row) {
    const int N = 1 << T.logN;
    FwdRow R;
    R.aux = nullptr;
    R.d0 = R.d1 = 0;
    if (LOAD == LOAD_MODUP) {
        const int r = row % T.nExt;
        const int j = (row / T.nExt) % T.beta;
        const int src = row / (T.nExt * T.beta);
        R.prime = r;
        R.out = a.out + (size_t)row * N;
        R.in = a.in + (size_t)src * a.in_stride;
        R.d0 = j * T.alpha;
        R.d1 = min(R.d0 + T.alpha, T.L);
    } else if (LOAD == LOAD_DELTA || LOAD == LOAD_DELTA_H) {
        const int i_q = row % T.L;
        const int slot = row / T.L;
        R.prime = i_q;
        R.out = a.out + (size_t)row * N;
        R.aux = a.aux + (size_t)slot * T.nExt * N + (size_t)i_q * N;
        R.in = a.in + (size_t)slot * a.in_stride;
    } else {
        const int g = row / a.per, rr = row % a.per;
        R.prime = a.prime_base + rr;
        R.out = a.out + (size_t)g * a.out_stride + (size_t)rr * N;
        R.in = (a.in_tab ? a.in_tab[g] : a.in + (size_t)g * a.in_stride) + a.in_offset + (size_t)rr * N;
    }
    return R;
}

// Input value at position i of the row (before any stage).
template <int LOAD>
__device__ __forceinline__ double fwd_load(const DevTables &T, const FwdRow &R, int i) {
    const int N = 1 << T.logN;
    if (LOAD == LOAD_MODUP) {
        const int r = R.prime;
        if (r >= R.d0 && r < R.d1) return gld(R.in)[(size_t)r * N + i];
        if (R.d1 - R.d0 == 1) {
            // one-prime digit: the centered residue itself is the lift
            return centerm(gld(R.in)[(size_t)R.d0 * N + i], T.qt[R.d0].x, T.qt[R.d0].y);
        }
        const double qr = T.qt[r].x, qir = T.qt[r].y;
        double acc = 0.0;
        for (int s = R.d0; s < R.d1; ++s) {
            const double qs = T.qt[s].x, qis = T.qt[s].y;
            const double ct = centerm(mulm(gld(R.in)[(size_t)s * N + i], T.mu_invhat[s], qs, qis), qs, qis);
            acc += mulm(ct, T.mu_hat[s * T.nExt + r], qr, qir);
        }
        return redm(acc, qr, qir);
    } else if (LOAD == LOAD_DELTA) {
        const int iq = R.prime;
        const double qr = T.qt[iq].x, qir = T.qt[iq].y;
        if (T.alpha == 1) return mulm(gld(R.in)[i], T.md_hat[iq], qr, qir);
        double acc = 0.0;
        for (int k = 0; k < T.alpha; ++k) acc += mulm(gld(R.in)[(size_t)k * N + i], T.md_hat[k * T.L + iq], qr, qir);
        return redm(acc, qr, qir);
    } else {
        return gld(R.in)[i];
    }
}

// fwd_load of NB positions pos(0..NB-1).  The lift of a two-prime digit
// (LOAD_MODUP) or of two special primes (LOAD_DELTA) issues all its loads
// before the arithmetic: fwd_load's loop over a run-time prime count keeps
// them one position at a time.  The sums are the same, in the same order.
template <int LOAD, int NB, class Pos>
__device__ __forceinline__ void fwd_load_batch(const DevTables &T, const FwdRow &R, Pos pos, double *x) {
    const int N = 1 << T.logN;
    if (LOAD == LOAD_DELTA && T.alpha == 1) {
        const int iq = R.prime;
        const double q = T.qt[iq].x, qi = T.qt[iq].y, h = T.md_hat[iq];
        double v[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) v[b] = gld(R.in)[pos(b)];
#pragma unroll
        for (int b = 0; b < NB; ++b) x[b] = mulm(v[b], h, q, qi);
        return;
    }
    if (LOAD == LOAD_MODUP && R.d1 - R.d0 == 1) {
        // a one-prime digit: the row itself under its own prime, else its
        // centered residue
        const bool own = R.prime == R.d0;
        const double qd = T.qt[R.d0].x, qid = T.qt[R.d0].y;
        double v[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) v[b] = gld(R.in)[(size_t)R.d0 * N + pos(b)];
#pragma unroll
        for (int b = 0; b < NB; ++b) x[b] = own ? v[b] : centerm(v[b], qd, qid);
        return;
    }
    if (LOAD == LOAD_DELTA && T.alpha == 2) {
        const int iq = R.prime;
        const double q = T.qt[iq].x, qi = T.qt[iq].y;
        const double h0 = T.md_hat[iq], h1 = T.md_hat[T.L + iq];
        double v0[NB], v1[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int i = pos(b);
            v0[b] = gld(R.in)[i];
            v1[b] = gld(R.in)[N + i];
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            double acc = 0.0;
            acc += mulm(v0[b], h0, q, qi);
            acc += mulm(v1[b], h1, q, qi);
            x[b] = redm(acc, q, qi);
        }
        return;
    }
    if (LOAD == LOAD_MODUP && R.d1 - R.d0 == 2 && (R.prime < R.d0 || R.prime >= R.d1)) {
        const int r = R.prime, s0 = R.d0, s1 = R.d0 + 1;
        const double qr = T.qt[r].x, qir = T.qt[r].y;
        const double q0 = T.qt[s0].x, qi0 = T.qt[s0].y, q1 = T.qt[s1].x, qi1 = T.qt[s1].y;
        const double mi0 = T.mu_invhat[s0], mi1 = T.mu_invhat[s1];
        const double mh0 = T.mu_hat[s0 * T.nExt + r], mh1 = T.mu_hat[s1 * T.nExt + r];
        double v0[NB], v1[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int i = pos(b);
            v0[b] = gld(R.in)[(size_t)s0 * N + i];
            v1[b] = gld(R.in)[(size_t)s1 * N + i];
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            double acc = 0.0;
            acc += mulm(centerm(mulm(v0[b], mi0, q0, qi0), q0, qi0), mh0, qr, qir);
            acc += mulm(centerm(mulm(v1[b], mi1, q1, qi1), q1, qi1), mh1, qr, qir);
            x[b] = redm(acc, qr, qir);
        }
        return;
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) x[b] = fwd_load<LOAD>(T, R, pos(b));
}

// Final store of position i (after the last stage).
template <int LOAD>
__device__ __forceinline__ void fwd_store(const DevTables &T, const FwdRow &R, int i, double v, double q, double qi) {
    if (LOAD == LOAD_DELTA || LOAD == LOAD_DELTA_H) {
        // E = (U - delta) * P^-1: the finished, divided output of the job
        gst(R.out)[i] = mulm(gld(R.aux)[i] - v, T.pinv[R.prime], q, qi);
    } else {
        gst(R.out)[i] = v;
    }
}

struct InvRow {
    int prime, rr;
    double *out;
    const double *in;
};

__device__ __forceinline__ InvRow inv_row(const DevTables &T, const NttArgs &a, int row) {
    const int N = 1 << T.logN;
    InvRow R;
    const int g = row / a.per;
    R.rr = row % a.per;
    R.prime = a.prime_base + R.rr;
    R.out = a.out + (size_t)g * a.out_stride + (size_t)R.rr * N;
    R.in = (a.in_tab ? a.in_tab[g] : a.in + (size_t)g * a.in_stride) + a.in_offset + (size_t)R.rr * N;
    return R;
}

// The factor every inverse output of the row is multiplied by: N^-1, or for
// STORE_MDR the division's N^-1 t^-1 (P/p_k)^-1.  Read once per row: read in
// inv_store, the compiler would read it again after every store (it cannot
// tell the tables from the output row).
template <int STORE>
__device__ __forceinline__ double inv_factor(const DevTables &T, const InvRow &R) {
    return STORE == STORE_MDR ? T.md_coef[R.rr] : T.ninv[R.prime];
}

template <int STORE>
__device__ __forceinline__ void inv_store(const InvRow &R, int i, double v, double f, double q, double qi) {
    if (STORE == STORE_MDR) {
        gst(R.out)[i] = centerm(mulm(v, f, q, qi), q, qi);
    } else {
        double x = mulm(v, f, q, qi);
        if (STORE == STORE_CANON) x = canonm(centerm(x, q, qi), q);
        gst(R.out)[i] = x;
    }
}

// ---- one workgroup per row ----

// Workgroups of a launch go to the 8 XCDs (each with its own L2) in turn by
// index.  With xcd_rows set, workgroup w takes the row that makes each XCD's
// workgroups a contiguous block of rows, so rows that read the same input
// row (the L primes of a division slot, the nExt primes of a hoisted digit)
// share that XCD's L2.  A permutation of the rows: every row is still done
// once, by one workgroup.
constexpr int NUM_XCD = 8;
__device__ __forceinline__ int xcd_row(int w, int n) {
    const int x = w % NUM_XCD, k = w / NUM_XCD;
    const int per = n / NUM_XCD, extra = n % NUM_XCD;   // XCD x holds per + (x < extra) workgroups
    return x * per + min(x, extra) + k;
}

template <int LOAD, int LOGN, int RK = rk_of(LOGN)>
__global__ void __launch_bounds__(NTT_THREADS_MAX) __attribute__((amdgpu_waves_per_eu(waves_of(LOGN, RK))))
k_ntt_fwd(DevTables T, NttArgs a) {
    extern __shared__ double sh[];
    constexpr int N = 1 << LOGN;
    const int wrow = T.xcd_rows ? xcd_row((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
    const FwdRow R = fwd_row<LOAD>(T, a, wrow);
    const double *tw = T.twf + (size_t)R.prime * N;
    if constexpr (LOAD == LOAD_DELTA_H) {
        if constexpr (direct_rows<LOGN>()) {
            // the r rows hold the two halves of the special prime's inverse
            // before its last stage: apply that stage (pairs i, i + N/2), the
            // scaling and centering of STORE_MDR, then the lift of LOAD_DELTA
            using RW = Rows<LOGN, RK>;
            constexpr int HALF = 1 << (RW::RK - 1);
            const int pk = T.L;
            const double qp = T.qt[pk].x, qip = T.qt[pk].y, wl = T.twi[(size_t)pk * N + 1];
            const double cf = T.md_coef[0], hat = T.md_hat[R.prime];
            const double q = T.qt[R.prime].x, qi = T.qt[R.prime].y;
            double x[1 << RW::RK];
#pragma unroll
            for (int b = 0; b < HALF; ++b) {
                const int i = (int)threadIdx.x + b * RW::NT;
                const double A = gld(R.in)[i], B = gld(R.in)[i + N / 2];
                const double s0 = redm(A + B, qp, qip), d0 = mulm(A - B, wl, qp, qip);
                x[b] = mulm(centerm(mulm(s0, cf, qp, qip), qp, qip), hat, q, qi);
                x[b + HALF] = mulm(centerm(mulm(d0, cf, qp, qip), qp, qip), hat, q, qi);
            }
            const double pinv = T.pinv[R.prime];
            fwd_row_regs<LOGN, RK>(
                sh, tw, q, qi, x, [&](int i, double v, double u) { gst(R.out)[i] = mulm(u - v, pinv, q, qi); }, 0,
                [&](int i) { return gld(R.aux)[i]; });
        }
    } else if constexpr (direct_rows<LOGN>()) {
        using RW = Rows<LOGN, RK>;
        const double q = T.qt[R.prime].x, qi = T.qt[R.prime].y;
        double x[1 << RW::RK];
        fwd_load_batch<LOAD, (1 << RW::RK)>(T, R, [&](int b) { return (int)threadIdx.x + b * RW::NT; }, x);
        if constexpr (LOAD == LOAD_DELTA) {
            // (U - delta) P^-1 with every U word loaded before the first store
            const double pinv = T.pinv[R.prime];
            fwd_row_regs<LOGN, RK>(
                sh, tw, q, qi, x, [&](int i, double v, double u) { gst(R.out)[i] = mulm(u - v, pinv, q, qi); }, 0,
                [&](int i) { return gld(R.aux)[i]; });
        } else {
            fwd_row_regs<LOGN, RK>(sh, tw, q, qi, x, [&](int i, double v, double) { gst(R.out)[i] = v; });
        }
    } else {
        for (int i = threadIdx.x; i < N; i += blockDim.x) sh[lds_ix(i)] = fwd_load<LOAD>(T, R, i);
        __syncthreads();
        const double q = T.qt[R.prime].x, qi = T.qt[R.prime].y;
        fwd_rows_c<LOGN, 0>(sh, tw, q, qi);
        for (int i = threadIdx.x; i < N; i += blockDim.x) fwd_store<LOAD>(T, R, i, sh[lds_ix(i)], q, qi);
    }
}

template <int STORE, int LOGN, int RK = rk_of(LOGN)>
__global__ void __launch_bounds__(NTT_THREADS_MAX) __attribute__((amdgpu_waves_per_eu(waves_of(LOGN, RK))))
k_ntt_inv(DevTables T, NttArgs a) {
    extern __shared__ double sh[];
    constexpr int N = 1 << LOGN;
    const InvRow R = inv_row(T, a, STORE == STORE_MDR_H ? blockIdx.x >> 1 : blockIdx.x);
    const double *tw = T.twi + (size_t)R.prime * N;
    if constexpr (STORE == STORE_MDR_H) {
        if constexpr (direct_rows<LOGN>() && RK >= 2) {
            // input half hh through the first logN - 1 stages, stored as is
            // (the consumer applies the last stage; see k_ntt_fwd), at the
            // row's radix on half as many threads (launched with N / 2^(RK+1)):
            // 4096-point halves in four radix-8 rounds rather than six
            // radix-4 rounds on twice the threads
            using RH = Rows<LOGN - 1, RK>;
            const int hh = blockIdx.x & 1;
            const double q = T.qt[R.prime].x, qi = T.qt[R.prime].y;
            double x[1 << RH::RK];
            inv_row_direct<LOGN - 1, RK, 1>(
                sh, tw, q, qi, [&](int i) { return gld(R.in)[(hh << (LOGN - 1)) + i]; }, x, hh);
#pragma unroll
            for (int b = 0; b < (1 << RH::RK); ++b)
                gst(R.out)[(hh << (LOGN - 1)) + (int)threadIdx.x + b * RH::NT] = x[b];
        }
        return;
    }
    if constexpr (direct_rows<LOGN>()) {
        using RW = Rows<LOGN, RK>;
        const double q = T.qt[R.prime].x, qi = T.qt[R.prime].y, f = inv_factor<STORE>(T, R);
        double x[1 << RW::RK];
        inv_row_direct<LOGN, RK>(sh, tw, q, qi, [&](int i) { return gld(R.in)[i]; }, x);
#pragma unroll
        for (int b = 0; b < (1 << RW::RK); ++b) inv_store<STORE>(R, (int)threadIdx.x + b * RW::NT, x[b], f, q, qi);
        return;
    }
    for (int i = threadIdx.x; i < N; i += blockDim.x) sh[lds_ix(i)] = gld(R.in)[i];
    __syncthreads();
    const double q = T.qt[R.prime].x, qi = T.qt[R.prime].y;
    inv_rows_c<LOGN, 0>(sh, tw, q, qi);
    const double f = inv_factor<STORE>(T, R);
    for (int i = threadIdx.x; i < N; i += blockDim.x) inv_store<STORE>(R, i, sh[lds_ix(i)], f, q, qi);
}

// ---- split rows: N = N1 x N2, N1 = 2^a (column length), N2 = 2^b ----
// Forward stages 0..a-1 pair elements of the same column {c + N2 j}; stages
// a..logN-1 pair elements of the same contiguous block of N2.  Each pass is
// one launch of SPLIT_ELEMS-element workgroups; the row goes through L2/HBM
// between them.  Used when few rows would leave most CUs idle, and for rows
// too long for one workgroup's LDS.

__device__ __forceinline__ void split_dims(int logN, int &a, int &b) {
    a = (logN + 1) >> 1;
    b = logN - a;
}

// LOGN > 0: a size known at compile time (rounds fully unrolled, twiddles
// preloaded); LOGN = 0: any size, runtime rounds.
// Column passes of 32768-point rows (256-point columns, 16 per workgroup,
// two radix-16 rounds) with both ends in registers: thread t owns column
// t % 16 and, in the first round, rows t / 16 + 16 b, in the second rows
// 16 (t / 16) + b, so every global access of a wave covers 16 adjacent
// columns (128 bytes) of 4 rows, and only the exchange between the rounds
// goes through LDS (one barrier instead of three).  The butterflies, twiddles
// and reductions are those of the staged rounds, so the values are the same.
constexpr int COL_LA = 8, COL_LB = 7, COL_W = SPLIT_ELEMS >> COL_LA;
static_assert(COL_W * 16 == SPLIT_THREADS, "one thread per (column, group) in each round");

template <int LOAD>
__device__ __forceinline__ void fwd_cols_direct(const DevTables &T, const FwdRow &R, int c0, double *sh) {
    const int sb = (int)threadIdx.x % COL_W, g = (int)threadIdx.x / COL_W;
    const double q = T.qt[R.prime].x, qi = T.qt[R.prime].y;
    const double *__restrict__ tw = T.twf + (size_t)R.prime * (1 << (COL_LA + COL_LB));
    double x[16], w[15];
    // round 1: stages 0..3 of the column, rows g + 16 b (group g of stride 16)
    fwd_load_batch<LOAD, 16>(T, R, [&](int b) { return c0 + sb + ((g + 16 * b) << COL_LB); }, x);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < (1 << u); ++c) w[(1 << u) - 1 + c] = tw[(1 << u) + c];
    fwd_bfly<COL_LA + COL_LB, 0, 4>(x, w, q, qi);
#pragma unroll
    for (int b = 0; b < 16; ++b) sh[lds_ix_step<16>((sb << COL_LA) + g, b)] = x[b];
    __syncthreads();
    // round 2: stages 4..7, rows 16 g + b (block g of the column)
#pragma unroll
    for (int b = 0; b < 16; ++b) x[b] = sh[lds_ix((sb << COL_LA) + (g << 4) + b)];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < (1 << u); ++c) w[(1 << u) - 1 + c] = tw[(1 << (4 + u)) + (g << u) + c];
    fwd_bfly<COL_LA + COL_LB, 4, 4>(x, w, q, qi);
#pragma unroll
    for (int b = 0; b < 16; ++b) gst(R.out)[c0 + sb + ((16 * g + b) << COL_LB)] = x[b];
}

template <int LOAD, int LOGN>
__global__ void __launch_bounds__(SPLIT_THREADS)
k_ntt_fwd_cols(DevTables T, NttArgs a) {
    __shared__ double sh[SPLIT_ELEMS + SPLIT_ELEMS / 16];
    const int logN = LOGN > 0 ? LOGN : T.logN;
    int la, lb;
    split_dims(logN, la, lb);
    const int N2 = 1 << lb;
    const int cw = SPLIT_ELEMS >> la;                // columns per workgroup
    const int wpr = N2 / cw;                         // workgroups per row
    const int row = blockIdx.x / wpr;
    const int c0 = (blockIdx.x % wpr) * cw;
    const FwdRow R = fwd_row<LOAD>(T, a, row);
    if constexpr (LOGN == COL_LA + COL_LB) {
        fwd_cols_direct<LOAD>(T, R, c0, sh);
        return;
    }
    for (int e = threadIdx.x; e < SPLIT_ELEMS; e += blockDim.x) {
        const int cc = e % cw, j = e / cw;
        sh[lds_ix((cc << la) + j)] = fwd_load<LOAD>(T, R, c0 + cc + (j << lb));
    }
    __syncthreads();
    const double q = T.qt[R.prime].x, qi = T.qt[R.prime].y;
    const double *tw = T.twf + (size_t)R.prime * (1 << logN);
    if constexpr (LOGN > 0) {
        constexpr int LA = (LOGN + 1) >> 1;
        fwd_stages_t<LA, (SPLIT_ELEMS >> LA), 0, 0, LOGN, true>(sh, tw, 1, 0, q, qi);
    } else {
        fwd_stages(sh, tw, la, cw, 0, 1, 0, 0, logN, true, q, qi);
    }
    for (int e = threadIdx.x; e < SPLIT_ELEMS; e += blockDim.x) {
        const int cc = e % cw, j = e / cw;
        gst(R.out)[c0 + cc + (j << lb)] = sh[lds_ix((cc << la) + j)];
    }
}

template <int LOAD, int LOGN>
__global__ void __launch_bounds__(SPLIT_THREADS)
k_ntt_fwd_blocks(DevTables T, NttArgs a) {
    __shared__ double sh[SPLIT_ELEMS + SPLIT_ELEMS / 16];
    const int logN = LOGN > 0 ? LOGN : T.logN;
    int la, lb;
    split_dims(logN, la, lb);
    const int N = 1 << logN;
    const int bw = SPLIT_ELEMS >> lb;                // blocks per workgroup
    const int wpr = N / SPLIT_ELEMS;
    const int row = blockIdx.x / wpr;
    const int off = (blockIdx.x % wpr) * SPLIT_ELEMS;
    const FwdRow R = fwd_row<LOAD>(T, a, row);
    const double q = T.qt[R.prime].x, qi = T.qt[R.prime].y;
    const int B0 = off >> lb;
    const double *tw = T.twf + (size_t)R.prime * N;
    if constexpr (LOGN == COL_LA + COL_LB) {
        // 128-point blocks, 32 per workgroup: the first radix-16 round
        // (stages 8..11) straight from memory, thread t on elements
        // 8 b + t mod 8 of block t / 8 (64-byte runs per access), the rest as
        // in the staged rounds
        const int sb = (int)threadIdx.x >> 3, low = (int)threadIdx.x & 7;
        const int C = (1 << COL_LA) + B0 + sb;
        double x[16], w[15];
#pragma unroll
        for (int b = 0; b < 16; ++b) x[b] = gld(R.out)[off + (sb << COL_LB) + low + 8 * b];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < (1 << u); ++c) w[(1 << u) - 1 + c] = tw[(C << u) + c];
        fwd_bfly<COL_LA + COL_LB, COL_LA, 4>(x, w, q, qi);
#pragma unroll
        for (int b = 0; b < 16; ++b) sh[lds_ix_step<8>((sb << COL_LB) + low, b)] = x[b];
        __syncthreads();
        fwd_stages_t<COL_LB, (SPLIT_ELEMS >> COL_LB), 4, COL_LA, LOGN, false>(sh, tw, (1 << COL_LA) + B0, 1, q, qi);
        for (int e = threadIdx.x; e < SPLIT_ELEMS; e += blockDim.x)
            fwd_store<LOAD>(T, R, off + e, sh[lds_ix(e)], q, qi);
        return;
    }
    for (int e = threadIdx.x; e < SPLIT_ELEMS; e += blockDim.x) sh[lds_ix(e)] = gld(R.out)[off + e];
    __syncthreads();
    if constexpr (LOGN > 0) {
        constexpr int LA = (LOGN + 1) >> 1, LB = LOGN - LA;
        fwd_stages_t<LB, (SPLIT_ELEMS >> LB), 0, LA, LOGN, false>(sh, tw, (1 << LA) + B0, 1, q, qi);
    } else {
        fwd_stages(sh, tw, lb, bw, 0, (1 << la) + B0, 1, la, logN, false, q, qi);
    }
    for (int e = threadIdx.x; e < SPLIT_ELEMS; e += blockDim.x) fwd_store<LOAD>(T, R, off + e, sh[lds_ix(e)], q, qi);
}

template <int LOGN>
__global__ void __launch_bounds__(SPLIT_THREADS)
k_ntt_inv_blocks(DevTables T, NttArgs a) {
    __shared__ double sh[SPLIT_ELEMS + SPLIT_ELEMS / 16];
    const int logN = LOGN > 0 ? LOGN : T.logN;
    int la, lb;
    split_dims(logN, la, lb);
    const int N = 1 << logN;
    const int bw = SPLIT_ELEMS >> lb;
    const int wpr = N / SPLIT_ELEMS;
    const int row = blockIdx.x / wpr;
    const int off = (blockIdx.x % wpr) * SPLIT_ELEMS;
    const InvRow R = inv_row(T, a, row);
    for (int e = threadIdx.x; e < SPLIT_ELEMS; e += blockDim.x) sh[lds_ix(e)] = gld(R.in)[off + e];
    __syncthreads();
    const double q = T.qt[R.prime].x, qi = T.qt[R.prime].y;
    const int B0 = off >> lb;
    const double *tw = T.twi + (size_t)R.prime * N;
    if constexpr (LOGN == COL_LA + COL_LB) {
        // 128-point blocks, 32 per workgroup: the first round (half-sizes
        // 1..8) in LDS, the last (16, 32, 64) straight to memory, each thread
        // on elements 16 b + g mod 16 of block g / 16 for its two groups g
        // (16 adjacent elements of 4 blocks per access)
        const int C0 = (1 << COL_LA) + B0;
        inv_round_t<4, COL_LB, (SPLIT_ELEMS >> COL_LB), 0>(sh, tw, C0, 1, q, qi);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int grp = (int)threadIdx.x + k * SPLIT_THREADS;
            const int sb = grp >> 4, low = grp & 15;
            double x[8], w[7];
            int wo = 0;
#pragma unroll
            for (int u = 0; u < 3; ++u) {
#pragma unroll
                for (int c = 0; c < (1 << (2 - u)); ++c) w[wo + c] = tw[((1 << COL_LB) >> (4 + u + 1)) * (C0 + sb) + c];
                wo += 1 << (2 - u);
            }
#pragma unroll
            for (int b = 0; b < 8; ++b) x[b] = sh[lds_ix_step<16>((sb << COL_LB) + low, b)];
            inv_bfly_red<3>(x, w, q, qi);
#pragma unroll
            for (int b = 0; b < 8; ++b) gst(R.out)[off + (sb << COL_LB) + low + 16 * b] = x[b];
        }
        return;
    }
    if constexpr (LOGN > 0) {
        constexpr int LA = (LOGN + 1) >> 1, LB = LOGN - LA;
        inv_stages_t<LB, (SPLIT_ELEMS >> LB), 0>(sh, tw, (1 << LA) + B0, 1, q, qi);
    } else {
        inv_stages(sh, tw, lb, bw, (1 << la) + B0, 1, q, qi);
    }
    for (int e = threadIdx.x; e < SPLIT_ELEMS; e += blockDim.x) gst(R.out)[off + e] = sh[lds_ix(e)];
}

// The inverse column pass of 32768-point rows with both ends in registers
// (see fwd_cols_direct): the first round takes rows 16 (t / 16) + b of
// column t % 16 straight from memory, the second stores rows t / 16 + 16 b.
template <int STORE>
__device__ __forceinline__ void inv_cols_direct(const DevTables &T, const InvRow &R, int c0, double *sh) {
    const int sb = (int)threadIdx.x % COL_W, g = (int)threadIdx.x / COL_W;
    const double q = T.qt[R.prime].x, qi = T.qt[R.prime].y, f = inv_factor<STORE>(T, R);
    const double *__restrict__ tw = T.twi + (size_t)R.prime * (1 << (COL_LA + COL_LB));
    double x[16], w[15];
    // round 1: half-sizes 1..8, rows 16 g + b (block g of the column)
#pragma unroll
    for (int b = 0; b < 16; ++b) x[b] = gld(R.out)[c0 + sb + ((16 * g + b) << COL_LB)];
    {
        int wo = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int c = 0; c < (1 << (3 - u)); ++c)
                w[wo + c] = tw[((1 << COL_LA) >> (u + 1)) + (g << (3 - u)) + c];
            wo += 1 << (3 - u);
        }
    }
    inv_bfly_red<4>(x, w, q, qi);
#pragma unroll
    for (int b = 0; b < 16; ++b) sh[lds_ix((sb << COL_LA) + (g << 4) + b)] = x[b];
    __syncthreads();
    // round 2: half-sizes 16..128, rows g + 16 b
#pragma unroll
    for (int b = 0; b < 16; ++b) x[b] = sh[lds_ix_step<16>((sb << COL_LA) + g, b)];
    {
        int wo = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int c = 0; c < (1 << (3 - u)); ++c) w[wo + c] = tw[((1 << COL_LA) >> (4 + u + 1)) + c];
            wo += 1 << (3 - u);
        }
    }
    inv_bfly_red<4>(x, w, q, qi);
#pragma unroll
    for (int b = 0; b < 16; ++b) inv_store<STORE>(R, c0 + sb + ((g + 16 * b) << COL_LB), x[b], f, q, qi);
}

template <int STORE, int LOGN>
__global__ void __launch_bounds__(SPLIT_THREADS)
k_ntt_inv_cols(DevTables T, NttArgs a) {
    __shared__ double sh[SPLIT_ELEMS + SPLIT_ELEMS / 16];
    const int logN = LOGN > 0 ? LOGN : T.logN;
    int la, lb;
    split_dims(logN, la, lb);
    const int N2 = 1 << lb;
    const int cw = SPLIT_ELEMS >> la;
    const int wpr = N2 / cw;
    const int row = blockIdx.x / wpr;
    const int c0 = (blockIdx.x % wpr) * cw;
    const InvRow R = inv_row(T, a, row);
    if constexpr (LOGN == COL_LA + COL_LB) {
        inv_cols_direct<STORE>(T, R, c0, sh);
        return;
    }
    for (int e = threadIdx.x; e < SPLIT_ELEMS; e += blockDim.x) {
        const int cc = e % cw, j = e / cw;
        sh[lds_ix((cc << la) + j)] = gld(R.out)[c0 + cc + (j << lb)];
    }
    __syncthreads();
    const double q = T.qt[R.prime].x, qi = T.qt[R.prime].y;
    const double *tw = T.twi + (size_t)R.prime * (1 << logN);
    if constexpr (LOGN > 0) {
        constexpr int LA = (LOGN + 1) >> 1;
        inv_stages_t<LA, (SPLIT_ELEMS >> LA), 0>(sh, tw, 1, 0, q, qi);
    } else {
        inv_stages(sh, tw, la, cw, 1, 0, q, qi);
    }
    const double f = inv_factor<STORE>(T, R);
    for (int e = threadIdx.x; e < SPLIT_ELEMS; e += blockDim.x) {
        const int cc = e % cw, j = e / cw;
        inv_store<STORE>(R, c0 + cc + (j << lb), sh[lds_ix((cc << la) + j)], f, q, qi);
    }
}

// ---- fused chains for passes with few rows (single-prime digits) ----

// Hoisting, one workgroup per lifted row (src, digit j, prime r): the
// evaluation-form row j of the source's c1 is inverse-transformed, centered
// (the digit lift of a one-prime digit) and forward-transformed under prime
// r, all in LDS.  Row r = j is the source row itself.
// The row of workgroup `wg`: (source, digit j, prime r), and with SPLIT the
// half of the forward transform it finishes (two workgroups per row).
template <int SPLIT>
__device__ __forceinline__ void hoist_row(const DevTables &T, int wg, int &row, int &hh, int &r, int &j, int &src) {
    row = SPLIT ? wg >> 1 : wg;
    hh = SPLIT ? (wg & 1) : -1;
    r = row % T.nExt;
    j = (row / T.nExt) % T.beta;
    src = row / (T.nExt * T.beta);
}

template <int LOGN, int RK, int SPLIT>
__device__ __forceinline__ void hoist_body(const DevTables &T, double *y, const double *c1, int row, int hh, int r,
                                           int j, double *sh);

template <int LOGN, int RK = rk_of(LOGN), int SPLIT = 0>
__global__ void __launch_bounds__(NTT_THREADS_MAX) __attribute__((amdgpu_waves_per_eu(waves_of(LOGN, RK))))
k_hoist_fused(DevTables T, double *y, const double *const *srcs) {
    extern __shared__ double sh[];
    int row, hh, r, j, src;
    hoist_row<SPLIT>(T, (int)blockIdx.x, row, hh, r, j, src);
    hoist_body<LOGN, RK, SPLIT>(T, y, srcs[src], row, hh, r, j, sh);
}

// The same with the sources by value; workgroups past the hoist's copy a
// call's descriptor tables out of pinned host memory meanwhile.
template <int LOGN, int RK = rk_of(LOGN), int SPLIT = 0>
__global__ void __launch_bounds__(NTT_THREADS_MAX) __attribute__((amdgpu_waves_per_eu(waves_of(LOGN, RK))))
k_hoist_fused_copy(DevTables T, double *y, HoistSrc a) {
    extern __shared__ double sh[];
    const int hoist_wgs = (int)gridDim.x - a.copy_wgs;
    if ((int)blockIdx.x >= hoist_wgs) {
        const size_t stride = (size_t)a.copy_wgs * blockDim.x;
        for (size_t i = (size_t)(blockIdx.x - hoist_wgs) * blockDim.x + threadIdx.x; i < a.copy_n; i += stride)
            a.copy_dst[i] = a.copy_src[i];
        return;
    }
    int row, hh, r, j, src;
    hoist_row<SPLIT>(T, (int)blockIdx.x, row, hh, r, j, src);
    hoist_body<LOGN, RK, SPLIT>(T, y, a.p[src], row, hh, r, j, sh);
}

// The same with the sources by value and no copy.
template <int LOGN, int RK = rk_of(LOGN), int SPLIT = 0>
__global__ void __launch_bounds__(NTT_THREADS_MAX) __attribute__((amdgpu_waves_per_eu(waves_of(LOGN, RK))))
k_hoist_fused_v(DevTables T, double *y, HoistSrc a) {
    extern __shared__ double sh[];
    int row, hh, r, j, src;
    hoist_row<SPLIT>(T, (int)blockIdx.x, row, hh, r, j, src);
    hoist_body<LOGN, RK, SPLIT>(T, y, a.p[src], row, hh, r, j, sh);
}

template <int LOGN, int RK, int SPLIT>
__device__ __forceinline__ void hoist_body(const DevTables &T, double *y, const double *c1, int row, int hh, int r,
                                           int j, double *sh) {
    constexpr int N = 1 << LOGN;
    const double *c = c1 + (size_t)j * N;
    double *out = y + (size_t)row * N;
    if (r == j) {
        const int i0 = hh < 0 ? 0 : hh * (N / 2), i1 = hh < 0 ? N : i0 + N / 2;
        for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) gst(out)[i] = gld(c)[i];
        return;
    }
    const double *twj = T.twi + (size_t)j * N;
    if constexpr (direct_rows<LOGN>()) {
        using RW = Rows<LOGN, RK>;
        const double qj = T.qt[j].x, qij = T.qt[j].y, nj = T.ninv[j];
        double x[1 << RW::RK];
        inv_row_direct<LOGN, RK>(sh, twj, qj, qij, [&](int i) { return gld(c)[i]; }, x);
#pragma unroll
        for (int b = 0; b < (1 << RW::RK); ++b) x[b] = centerm(mulm(x[b], nj, qj, qij), qj, qij);
        const double q = T.qt[r].x, qi = T.qt[r].y;
        const auto st = [&](int i, double v, double) { gst(out)[i] = v; };
        if constexpr (SPLIT && RK >= 2)
            fwd_row_regs_half<LOGN, RK>(sh, T.twf + (size_t)r * N, q, qi, x, st, hh);
        else
            fwd_row_regs<LOGN, RK>(sh, T.twf + (size_t)r * N, q, qi, x, st);
        return;
    }
    for (int i = threadIdx.x; i < N; i += blockDim.x) sh[lds_ix(i)] = gld(c)[i];
    __syncthreads();
    const double qj = T.qt[j].x, qij = T.qt[j].y;
    inv_rows_c<LOGN, 0>(sh, twj, qj, qij);
    const double *twr = T.twf + (size_t)r * N;
    const double nj = T.ninv[j];
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const int x = lds_ix(i);
        sh[x] = centerm(mulm(sh[x], nj, qj, qij), qj, qij);
    }
    __syncthreads();
    const double q = T.qt[r].x, qi = T.qt[r].y;
    fwd_rows_c<LOGN, 0>(sh, twr, q, qi);
    for (int i = threadIdx.x; i < N; i += blockDim.x) gst(out)[i] = sh[lds_ix(i)];
}

// Division by P for one special prime, one workgroup per output row
// (slot, i): inverse transform of U's special row, exact centered r,
// delta_i = t (P/p) r mod q_i, forward transform, E_i = (U_i - delta_i) P^-1,
// written to E or (outs given) straight into the job's output ciphertext.
// (Giving a workgroup several primes of a slot, to share the inverse
// transform, was measured slower at 8192 points: one 135 KB workgroup per CU
// running three transforms against two 70 KB workgroups running two.)
template <int LOGN, int RK = rk_of(LOGN), int SPLIT = 0>
__global__ void __launch_bounds__(NTT_THREADS_MAX) __attribute__((amdgpu_waves_per_eu(waves_of(LOGN, RK))))
k_moddown_fused(DevTables T, double *E, const double *U, double *const *outs) {
    extern __shared__ double sh[];
    constexpr int N = 1 << LOGN;
    const int row = SPLIT ? blockIdx.x >> 1 : blockIdx.x;
    const int hh = SPLIT ? (int)(blockIdx.x & 1) : -1;   // the half of the forward transform (SPLIT)
    const int iq = row % T.L;
    const int slot = row / T.L;
    const double *u = U + (size_t)slot * T.nExt * N;
    const int pk = T.L;   // the special prime's index
    const double *twp = T.twi + (size_t)pk * N;
    if constexpr (direct_rows<LOGN>()) {
        using RW = Rows<LOGN, RK>;
        const double qp = T.qt[pk].x, qip = T.qt[pk].y;
        const double q = T.qt[iq].x, qi = T.qt[iq].y;
        const double cf = T.md_coef[0], h = T.md_hat[iq], pinv = T.pinv[iq];
        double x[1 << RW::RK];
        inv_row_direct<LOGN, RK>(sh, twp, qp, qip, [&](int i) { return gld(u)[(size_t)pk * N + i]; }, x);
#pragma unroll
        for (int b = 0; b < (1 << RW::RK); ++b) x[b] = mulm(centerm(mulm(x[b], cf, qp, qip), qp, qip), h, q, qi);
        const double *ui = u + (size_t)iq * N;
        double *out = outs ? outs[slot >> 1] + ((size_t)(slot & 1) * T.L + iq) * N : E + (size_t)row * N;
        const auto st = [&](int i, double v, double uw) { gst(out)[i] = mulm(uw - v, pinv, q, qi); };
        const auto pre = [&](int i) { return gld(ui)[i]; };
        if constexpr (SPLIT && RK >= 2)
            fwd_row_regs_half<LOGN, RK>(sh, T.twf + (size_t)iq * N, q, qi, x, st, hh, pre);
        else
            fwd_row_regs<LOGN, RK>(sh, T.twf + (size_t)iq * N, q, qi, x, st, 0, pre);
        return;
    }
    for (int i = threadIdx.x; i < N; i += blockDim.x) sh[lds_ix(i)] = u[(size_t)pk * N + i];
    __syncthreads();
    const double qp = T.qt[pk].x, qip = T.qt[pk].y;
    inv_rows_c<LOGN, 0>(sh, twp, qp, qip);
    const double *twq = T.twf + (size_t)iq * N;
    const double q = T.qt[iq].x, qi = T.qt[iq].y;
    const double cf = T.md_coef[0], h = T.md_hat[iq];
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const int x = lds_ix(i);
        const double rk = centerm(mulm(sh[x], cf, qp, qip), qp, qip);
        sh[x] = mulm(rk, h, q, qi);
    }
    __syncthreads();
    fwd_rows_c<LOGN, 0>(sh, twq, q, qi);
    const double pinv = T.pinv[iq];
    const double *ui = u + (size_t)iq * N;
    double *out = outs ? outs[slot >> 1] + ((size_t)(slot & 1) * T.L + iq) * N : E + (size_t)row * N;
    for (int i = threadIdx.x; i < N; i += blockDim.x) gst(out)[i] = mulm(gld(ui)[i] - sh[lds_ix(i)], pinv, q, qi);
}

// Radix exponent the row kernels of 2^logn points run with.
int row_rk(const DevTables &T, int logn) { return (logn == 12 || logn == 13) && T.row_rk ? T.row_rk : rk_of(logn); }

int ntt_threads(const DevTables &T) {
    const int N = T.N;
    int t = N >> row_rk(T, T.logN);
    if (t < 64) t = 64;
    if (t > NTT_THREADS_MAX) t = NTT_THREADS_MAX;
    return t;
}

size_t ntt_lds_bytes(int N) { return (size_t)(N + N / 16) * sizeof(double); }

bool use_split(const DevTables &T, int rows) {
    if (T.N > 16384) return true;
    return T.N >= 2 * SPLIT_ELEMS && rows < T.split_rows;
}

// Dispatch on log2 N for the compile-time-size kernels.
#define HG_LOGN_SWITCH(LN, CALL) \
    switch (LN) {                 \
        case 6: CALL(6); break;   \
        case 7: CALL(7); break;   \
        case 8: CALL(8); break;   \
        case 9: CALL(9); break;   \
        case 10: CALL(10); break; \
        case 11: CALL(11); break; \
        case 12: CALL(12); break; \
        case 13: CALL(13); break; \
        case 14: CALL(14); break; \
        default: break;           \
    }

// The same with the row radix: CALL(LN, RK) for the radix row_rk(LN).
#define HG_LOGN_RK_SWITCH(LN, CALL)                                  \
    switch (LN) {                                                    \
        case 6: CALL(6, rk_of(6)); break;                            \
        case 7: CALL(7, rk_of(7)); break;                            \
        case 8: CALL(8, rk_of(8)); break;                            \
        case 9: CALL(9, rk_of(9)); break;                            \
        case 10: CALL(10, rk_of(10)); break;                         \
        case 11: CALL(11, rk_of(11)); break;                         \
        case 12: if (row_rk(T, 12) == 4) { CALL(12, 4); } else { CALL(12, 3); } break; \
        case 13: if (row_rk(T, 13) == 4) { CALL(13, 4); } else { CALL(13, 3); } break; \
        case 14: CALL(14, rk_of(14)); break;                         \
        default: break;                                              \
    }

template <int LN, int RK>
void set_lds_attrs() {
    const int lds = 160 * 1024;
    (void)hipFuncSetAttribute((const void *)k_ntt_fwd<LOAD_PLAIN, LN, RK>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void *)k_ntt_fwd<LOAD_MODUP, LN, RK>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void *)k_ntt_fwd<LOAD_DELTA, LN, RK>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void *)k_ntt_inv<STORE_PLAIN, LN, RK>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void *)k_ntt_inv<STORE_MDR, LN, RK>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void *)k_ntt_inv<STORE_CANON, LN, RK>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void *)k_hoist_fused<LN, RK, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void *)k_moddown_fused<LN, RK, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void *)k_hoist_fused<LN, RK, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void *)k_hoist_fused_copy<LN, RK, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void *)k_hoist_fused_copy<LN, RK, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void *)k_hoist_fused_v<LN, RK, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void *)k_hoist_fused_v<LN, RK, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void *)k_moddown_fused<LN, RK, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void *)k_ntt_fwd<LOAD_DELTA_H, LN, RK>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void *)k_ntt_inv<STORE_MDR_H, LN, RK>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

}  // namespace

void kernels_init() {
#define HG_INIT(LN) set_lds_attrs<LN, rk_of(LN)>()
    for (int ln = 6; ln <= 14; ++ln) HG_LOGN_SWITCH(ln, HG_INIT)
#undef HG_INIT
    set_lds_attrs<12, 4>();
    set_lds_attrs<13, 4>();
}

int ntt_radix_rk(int radix) {
    if (radix != 0 && radix != 8 && radix != 16) throw std::invalid_argument("row radix must be 0, 8 or 16");
    return radix == 8 ? 3 : radix == 16 ? 4 : 0;
}

// A launch whose start and stop timestamps land in ev0 / ev1 (taken by the
// dispatch itself), or a plain launch.
template <typename... Args, typename F = void (*)(Args...)>
static void launch_ev(F kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1,
                      Args... args) {
    if (ev0 || ev1) hipExtLaunchKernelGGL(kernel, grid, block, lds, s, ev0, ev1, 0, args...);
    else hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
}

void ntt_fwd(const DevTables &T, NttLoad mode, const NttArgs &a, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (a.rows <= 0) return;
    if (use_split(T, a.rows)) {
        if (ev0) (void)hipEventRecord(ev0, s);   // a failed record surfaces when the timing is read
        dim3 grid((unsigned)(a.rows * (T.N / SPLIT_ELEMS))), block(SPLIT_THREADS);
#define HG_SPLIT_FWD(LN)                                                                                             \
    switch (mode) {                                                                                                 \
        case LOAD_MODUP: hipLaunchKernelGGL((k_ntt_fwd_cols<LOAD_MODUP, LN>), grid, block, 0, s, T, a);             \
                         hipLaunchKernelGGL((k_ntt_fwd_blocks<LOAD_MODUP, LN>), grid, block, 0, s, T, a); break;    \
        case LOAD_DELTA: hipLaunchKernelGGL((k_ntt_fwd_cols<LOAD_DELTA, LN>), grid, block, 0, s, T, a);             \
                         hipLaunchKernelGGL((k_ntt_fwd_blocks<LOAD_DELTA, LN>), grid, block, 0, s, T, a); break;    \
        default: hipLaunchKernelGGL((k_ntt_fwd_cols<LOAD_PLAIN, LN>), grid, block, 0, s, T, a);                     \
                 hipLaunchKernelGGL((k_ntt_fwd_blocks<LOAD_PLAIN, LN>), grid, block, 0, s, T, a); break;            \
    }
        if (T.logN == 15) { HG_SPLIT_FWD(15) } else { HG_SPLIT_FWD(0) }
#undef HG_SPLIT_FWD
        if (ev1) (void)hipEventRecord(ev1, s);
        return;
    }
    const size_t lds = ntt_lds_bytes(T.N);
    dim3 grid(a.rows), block(ntt_threads(T));
#define HG_FWD(LN, RK)                                                                                        \
    switch (mode) {                                                                                          \
        case LOAD_MODUP: launch_ev(k_ntt_fwd<LOAD_MODUP, LN, RK>, grid, block, lds, s, ev0, ev1, T, a); break;  \
        case LOAD_DELTA:                                                                                     \
            if (a.halves)                                                                                    \
                launch_ev(k_ntt_fwd<LOAD_DELTA_H, LN, RK>, grid, block, lds, s, ev0, ev1, T, a);             \
            else                                                                                             \
                launch_ev(k_ntt_fwd<LOAD_DELTA, LN, RK>, grid, block, lds, s, ev0, ev1, T, a);               \
            break;                                                                                           \
        default: launch_ev(k_ntt_fwd<LOAD_PLAIN, LN, RK>, grid, block, lds, s, ev0, ev1, T, a); break;          \
    }
    HG_LOGN_RK_SWITCH(T.logN, HG_FWD)
#undef HG_FWD
}

void ntt_inv(const DevTables &T, NttStore mode, const NttArgs &a, hipStream_t s) {
    if (a.rows <= 0) return;
    if (use_split(T, a.rows)) {
        dim3 grid((unsigned)(a.rows * (T.N / SPLIT_ELEMS))), block(SPLIT_THREADS);
#define HG_SPLIT_INV(LN)                                                                                          \
    hipLaunchKernelGGL((k_ntt_inv_blocks<LN>), grid, block, 0, s, T, a);                                          \
    switch (mode) {                                                                                              \
        case STORE_MDR: hipLaunchKernelGGL((k_ntt_inv_cols<STORE_MDR, LN>), grid, block, 0, s, T, a); break;     \
        case STORE_CANON: hipLaunchKernelGGL((k_ntt_inv_cols<STORE_CANON, LN>), grid, block, 0, s, T, a); break; \
        default: hipLaunchKernelGGL((k_ntt_inv_cols<STORE_PLAIN, LN>), grid, block, 0, s, T, a); break;          \
    }
        if (T.logN == 15) { HG_SPLIT_INV(15) } else { HG_SPLIT_INV(0) }
#undef HG_SPLIT_INV
        return;
    }
    const size_t lds = ntt_lds_bytes(T.N);
    const int halves = mode == STORE_MDR && a.halves ? 1 : 0;   // two workgroups per row, each half the threads
    dim3 grid(a.rows << halves), block(ntt_threads(T) >> halves);
#define HG_INV(LN, RK)                                                                                          \
    switch (mode) {                                                                                            \
        case STORE_MDR:                                                                                        \
            if (a.halves)                                                                                      \
                hipLaunchKernelGGL((k_ntt_inv<STORE_MDR_H, LN, RK>), grid, block, lds, s, T, a);               \
            else                                                                                               \
                hipLaunchKernelGGL((k_ntt_inv<STORE_MDR, LN, RK>), grid, block, lds, s, T, a);                 \
            break;                                                                                             \
        case STORE_CANON: hipLaunchKernelGGL((k_ntt_inv<STORE_CANON, LN, RK>), grid, block, lds, s, T, a); break; \
        default: hipLaunchKernelGGL((k_ntt_inv<STORE_PLAIN, LN, RK>), grid, block, lds, s, T, a); break;         \
    }
    HG_LOGN_RK_SWITCH(T.logN, HG_INV)
#undef HG_INV
}

bool fused_ok(const DevTables &T) { return T.alpha == 1 && T.N <= 16384; }

// Few-row chains (at most T.half_rows rows, one-workgroup rows only) run two
// workgroups per row, each finishing half of the forward transform.
static bool half_split(const DevTables &T, int rows) {
    return T.half_rows > 0 && rows <= T.half_rows && T.logN >= 10 && T.logN <= 14;
}

bool ntt_halves_ok(const DevTables &T, int rows) {
    return T.alpha == 1 && half_split(T, rows) && T.split_rows == 0;
}

void hoist_fused(const DevTables &T, double *y, const double *const *srcs, int nsrc, hipStream_t s) {
    if (nsrc <= 0) return;
    const int rows = nsrc * T.beta * T.nExt;
    const int split = half_split(T, rows) ? 1 : 0;
#define HG_HF(LN, RK)                                                                                           \
    if (split)                                                                                                  \
        hipLaunchKernelGGL((k_hoist_fused<LN, RK, 1>), dim3(rows << 1), dim3(ntt_threads(T)), ntt_lds_bytes(T.N), \
                           s, T, y, srcs);                                                                     \
    else                                                                                                        \
        hipLaunchKernelGGL((k_hoist_fused<LN, RK, 0>), dim3(rows), dim3(ntt_threads(T)), ntt_lds_bytes(T.N), s, T, \
                           y, srcs)
    HG_LOGN_RK_SWITCH(T.logN, HG_HF)
#undef HG_HF
}

bool hoist_copy_ok(int nsrc, size_t copy_bytes) {
    return nsrc > 0 && nsrc <= HOIST_MAX_SRC && copy_bytes % 16 == 0 && copy_bytes / 16 <= HOIST_MAX_COPY;
}

void hoist_fused_copy(const DevTables &T, double *y, const HoistSrc &a, int nsrc, hipStream_t s, hipEvent_t done) {
    if (!hoist_copy_ok(nsrc, a.copy_n * 16) || a.copy_wgs < 1)
        throw std::invalid_argument("hoist_fused_copy: sources or copy outside the launch's range");
    const int rows = nsrc * T.beta * T.nExt;
    const int split = half_split(T, rows) ? 1 : 0;
    const dim3 grid((unsigned)((rows << split) + a.copy_wgs)), block(ntt_threads(T));
#define HG_HFC(LN, RK)                                                                                 \
    if (split)                                                                                         \
        launch_ev(k_hoist_fused_copy<LN, RK, 1>, grid, block, ntt_lds_bytes(T.N), s, nullptr, done, T, y, a); \
    else                                                                                               \
        launch_ev(k_hoist_fused_copy<LN, RK, 0>, grid, block, ntt_lds_bytes(T.N), s, nullptr, done, T, y, a)
    HG_LOGN_RK_SWITCH(T.logN, HG_HFC)
#undef HG_HFC
}

void hoist_fused_v(const DevTables &T, double *y, const HoistSrc &a, int nsrc, hipStream_t s) {
    if (nsrc <= 0) return;
    if (nsrc > HOIST_MAX_SRC) throw std::invalid_argument("hoist_fused_v: more sources than a launch takes");
    const int rows = nsrc * T.beta * T.nExt;
    const int split = half_split(T, rows) ? 1 : 0;
    const dim3 grid((unsigned)(rows << split)), block(ntt_threads(T));
#define HG_HFV(LN, RK)                                                                                          \
    if (split)                                                                                                  \
        hipLaunchKernelGGL((k_hoist_fused_v<LN, RK, 1>), grid, block, ntt_lds_bytes(T.N), s, T, y, a);          \
    else                                                                                                        \
        hipLaunchKernelGGL((k_hoist_fused_v<LN, RK, 0>), grid, block, ntt_lds_bytes(T.N), s, T, y, a)
    HG_LOGN_RK_SWITCH(T.logN, HG_HFV)
#undef HG_HFV
}

void moddown_fused(const DevTables &T, double *E, const double *U, int nslots, hipStream_t s, double *const *outs) {
    if (nslots <= 0) return;
    const int rows = nslots * T.L;
    const int split = half_split(T, rows) ? 1 : 0;
#define HG_MF(LN, RK)                                                                                           \
    if (split)                                                                                                  \
        hipLaunchKernelGGL((k_moddown_fused<LN, RK, 1>), dim3(rows << 1), dim3(ntt_threads(T)), ntt_lds_bytes(T.N), \
                           s, T, E, U, outs);                                                                  \
    else                                                                                                        \
        hipLaunchKernelGGL((k_moddown_fused<LN, RK, 0>), dim3(rows), dim3(ntt_threads(T)), ntt_lds_bytes(T.N), s, \
                           T, E, U, outs)
    HG_LOGN_RK_SWITCH(T.logN, HG_MF)
#undef HG_MF
}

}  // namespace hg
