// HIP kernels for gfx950: negacyclic transforms, digit lifting, key-switch
// inner products, the division by P, tensor accumulation, sampling.
#include "kernels.h"

#include <hip/hip_ext.h>

#include <algorithm>
#include <stdexcept>

#include "arith.h"
#include "dev_common.h"
#include "gauss_cdt.h"

namespace hg {

namespace {

constexpr int EW_THREADS = 256;

constexpr int IP_THREADS = 256;

constexpr int MAX_GRID_Z = 65535;   // launches with more z blocks are split

__device__ __forceinline__ uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t sm_draw(uint64_t s0, uint64_t k) {
    return sm_mix(s0 + (k + 1) * 0x9E3779B97F4A7C15ULL);
}

// A switching key's a_j at evaluation position p of prime row r: the digit
// stream's draw r N + i, i = bitrev(p) the natural index of the evaluation
// point at position p, scaled into [0, q) by the high word of draw * q.
__device__ __forceinline__ double key_a(uint64_t stream, int r, int p, int logN, double q) {
    const uint64_t k = ((uint64_t)r << logN) + (uint64_t)brev_bits(p, logN);
    return (double)__umul64hi(sm_draw(stream, k), (uint64_t)q);
}

// Two consecutive words read once per launch (key and mask streams): a
// non-temporal load, so that the stream does not evict the hoisted digits
// and ciphertext rows that every job gathers from L2.
typedef double dvec2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_stream2(const double *p) {
    const dvec2 v = __builtin_nontemporal_load(gld((const dvec2 *)p));
    return make_double2(v.x, v.y);
}

// Two consecutive words through global (not flat) instructions.
__device__ __forceinline__ double2 ld2(const double *p) {
    const dvec2 v = *gld((const dvec2 *)p);
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ void st2(double *p, double2 v) {
    dvec2 w;
    w.x = v.x;
    w.y = v.y;
    *gst((dvec2 *)p) = w;
}

// The digit sums of the inner products add BETA products of |x| < 0.875 q
// (arith.h) before one reduction; with q < 2^50 that stays below 2^53, where
// FP64 holds every integer exactly, for up to 9 terms.  Longer sums (BETA up
// to 12) are reduced after every 8th term (then below q/2 + 1 + 7 q).
#define IP_REDUCE_AFTER(j, BETA) ((BETA) > 9 && ((j) & 7) == 7 && (j) + 1 < (BETA))

// Key-switching inner products with the automorphism folded into the gather
// of the hoisted digits; two consecutive positions per thread (16-byte key
// loads), the digit loop unrolled (BETA digits) so that all key loads of a
// term are in flight together.  grid: (N / 512, nExt, jobs).
// TAG names the launch for profilers (0: the eps/omega transform pass,
// 1: relinearisation, fold and single-ciphertext passes; the code is the
// same) and selects the load of keys and masks: non-temporal (0, 1: each
// word is read once per launch), or through the caches (2: a transform pass
// whose terms share keys, its jobs started in key order).  TAG 3: the
// launch's single job and its terms come by value in `one` (ip_one_launch)
// and the tables are not read; keys and masks load as with TAG 1.  TAG 4:
// the same for a relinearisation job, whose two terms are known.
template <int BETA, int TAG>
__device__ __forceinline__ void ip_body(const DevTables &T, double *U, const double *y, const double *const *keys,
                                        const uint64_t *streams, const double *const *masks, const IpJob *jobs,
                                        const IpTerm *terms, const IpOne &one) {
    const int N = 1 << T.logN;
    const int p = 2 * (blockIdx.x * blockDim.x + threadIdx.x);
    const int r = blockIdx.y;
    const int job = blockIdx.z;
    if (p >= N) return;
    const double q = T.qt[r].x, qi = T.qt[r].y;
    const size_t plane = (size_t)T.nExt * N;   // one digit (or component) of all primes
    const IpJob J = TAG >= 3 ? one.J : jobs[job];
    const bool qrow = r < T.L;
    double a0x = 0.0, a0y = 0.0, a1x = 0.0, a1y = 0.0;   // key-switched sums
    double c0x = 0.0, c0y = 0.0, c1x = 0.0, c1y = 0.0;   // unswitched sums (ciphertext primes)
    // one term: its mask (mbase, when tm.mask >= 0), key b half (kbase) and
    // a-half streams (ks, both when tm.kind != IP_PLAIN)
    const auto term = [&](const IpTerm &tm, const double *mbase, const double *kbase, const uint64_t *ks) {
        double2 mv = make_double2(1.0, 1.0);
        if (tm.mask >= 0) {
            const double *mrow = mbase + (size_t)r * N + p;
            mv = TAG == 2 ? ld2(mrow) : ld_stream2(mrow);
        }
        // positions p, p + 1 (p even) gather from the aligned pair {pb, pb + 1}
        // (the automorphism flips bit 0 of the source with bit 0 of p), in
        // swapped order when sw
        const int pp = tm.g == 1 ? p : perm_index(p, tm.g, T.logN);
        const int pb = pp & ~1;
        const bool sw = pp & 1;
        if (tm.kind != IP_PLAIN) {
            const double *ys = y + (size_t)J.src * BETA * plane + (size_t)r * N;
            const double *kb = kbase + (size_t)r * N + p;
            double y0[BETA], y1[BETA];
            double2 kbv[BETA], kav[BETA];
#pragma unroll
            for (int j = 0; j < BETA; ++j) {
                const double2 v = ld2(ys + (size_t)j * plane + pb);
                y0[j] = sw ? v.y : v.x;
                y1[j] = sw ? v.x : v.y;
                kbv[j] = TAG == 2 ? ld2(kb + (size_t)j * plane) : ld_stream2(kb + (size_t)j * plane);
            }
#pragma unroll
            for (int j = 0; j < BETA; ++j)
                kav[j] = make_double2(key_a(ks[j], r, p, T.logN, q), key_a(ks[j], r, p + 1, T.logN, q));
            double s0x = 0.0, s0y = 0.0, s1x = 0.0, s1y = 0.0;
#pragma unroll
            for (int j = 0; j < BETA; ++j) {
                s0x += mulm(y0[j], kbv[j].x, q, qi);
                s0y += mulm(y1[j], kbv[j].y, q, qi);
                s1x += mulm(y0[j], kav[j].x, q, qi);
                s1y += mulm(y1[j], kav[j].y, q, qi);
                if (IP_REDUCE_AFTER(j, BETA)) {
                    s0x = redm(s0x, q, qi);
                    s0y = redm(s0y, q, qi);
                    s1x = redm(s1x, q, qi);
                    s1y = redm(s1y, q, qi);
                }
            }
            s0x = redm(s0x, q, qi);
            s0y = redm(s0y, q, qi);
            s1x = redm(s1x, q, qi);
            s1y = redm(s1y, q, qi);
            if (tm.mask >= 0) {
                s0x = mulm(s0x, mv.x, q, qi);
                s0y = mulm(s0y, mv.y, q, qi);
                s1x = mulm(s1x, mv.x, q, qi);
                s1y = mulm(s1y, mv.y, q, qi);
            }
            a0x = redm(a0x + s0x, q, qi);
            a0y = redm(a0y + s0y, q, qi);
            a1x = redm(a1x + s1x, q, qi);
            a1y = redm(a1y + s1y, q, qi);
        }
        if (qrow && tm.kind != IP_RELIN) {
            const double2 cv = ld2(J.c0 + (size_t)r * N + pb);
            double x0 = sw ? cv.y : cv.x, x1 = sw ? cv.x : cv.y;
            if (tm.mask >= 0) {
                x0 = mulm(x0, mv.x, q, qi);
                x1 = mulm(x1, mv.y, q, qi);
            }
            c0x = redm(c0x + x0, q, qi);
            c0y = redm(c0y + x1, q, qi);
            if (tm.g == 1) {
                const double2 w = ld2(J.c1 + (size_t)r * N + p);
                double z0 = w.x, z1 = w.y;
                if (tm.mask >= 0) {
                    z0 = mulm(z0, mv.x, q, qi);
                    z1 = mulm(z1, mv.y, q, qi);
                }
                c1x = redm(c1x + z0, q, qi);
                c1y = redm(c1y + z1, q, qi);
            }
        }
    };
    if constexpr (TAG == 4) {
        // a relinearisation: the unswitched, unmasked, unrotated term, then
        // the key switch of the hoisted c2, both known here, so that no
        // branch on a term's fields holds the second term's loads back
        term(IpTerm{1, -1, -1, IP_PLAIN}, nullptr, nullptr, nullptr);
        term(IpTerm{1, -1, 0, IP_RELIN}, nullptr, one.key, one.st);
    } else if constexpr (TAG == 3) {
#pragma unroll
        for (int u = 0; u < IP_ONE_MAX_TERMS; ++u)
            if (u < J.nt) term(one.tm[u], one.mask[u], one.key, one.st);
    } else {
        for (int tix = J.t0; tix < J.t0 + J.nt; ++tix) {
            const IpTerm tm = terms[tix];
            const bool ksw = tm.kind != IP_PLAIN;
            term(tm, tm.mask >= 0 ? masks[tm.mask] : nullptr, ksw ? keys[tm.key] : nullptr,
                 ksw ? streams + (size_t)tm.key * BETA : nullptr);
        }
    }
    if (qrow) {
        const double P = T.pmod[r];
        a0x = redm(a0x + mulm(c0x, P, q, qi), q, qi);
        a0y = redm(a0y + mulm(c0y, P, q, qi), q, qi);
        a1x = redm(a1x + mulm(c1x, P, q, qi), q, qi);
        a1y = redm(a1y + mulm(c1y, P, q, qi), q, qi);
    }
    double *u = U + (size_t)J.slot * 2 * plane + (size_t)r * N + p;
    *(double2 *)u = make_double2(a0x, a0y);
    *(double2 *)(u + plane) = make_double2(a1x, a1y);
}

template <int BETA, int TAG>
__global__ void __launch_bounds__(IP_THREADS)
k_ip(DevTables T, double *U, const double *y, const double *const *keys, const uint64_t *streams,
     const double *const *masks, const IpJob *jobs, const IpTerm *terms) {
    const IpOne none{};
    ip_body<BETA, TAG>(T, U, y, keys, streams, masks, jobs, terms, none);
}

template <int BETA, bool RELIN>
__global__ void __launch_bounds__(IP_THREADS) k_ip_one(DevTables T, double *U, const double *y, IpOne one) {
    ip_body<BETA, RELIN ? 4 : 3>(T, U, y, nullptr, nullptr, nullptr, nullptr, nullptr, one);
}

// Key-stationary inner products for batches.  The key-switched terms of a
// pass are split into rounds: round s holds the s-th key-switched term of
// every job that has one.  Within a round, terms that use the same key form
// chunks; one workgroup loads the chunk's key words at its positions once
// and applies them to every term of the chunk (each with its own job's
// hoisted digits and mask).  Round 0 also adds each job's unswitched part
// (P * masked c0 of every term, and c1 of unrotated terms) and writes U;
// later rounds add to U.  A job appears at most once per round, so no two
// workgroups of a launch write the same words.  tasks[i] = (job, term);
// chunks[c] = (first task, count), all of one key.
template <int BETA, int TAG>
__global__ void __launch_bounds__(IP_THREADS)
k_ip_keyed(DevTables T, double *U, const double *y, const double *const *keys, const uint64_t *streams,
           const double *const *masks, const IpJob *jobs, const IpTerm *terms, const int2 *chunks, const int2 *tasks,
           int first_round) {
    const int N = 1 << T.logN;
    const int p = 2 * (blockIdx.x * blockDim.x + threadIdx.x);
    const int r = blockIdx.y;
    if (p >= N) return;
    const double q = T.qt[r].x, qi = T.qt[r].y;
    const size_t plane = (size_t)T.nExt * N;
    const bool qrow = r < T.L;
    const int2 ch = chunks[blockIdx.z];
    double2 kb[BETA], ka[BETA];
    {
        const int key = terms[tasks[ch.x].y].key;
        const double *kp = keys[key] + (size_t)r * N + p;
        const uint64_t *ks = streams + (size_t)key * BETA;
#pragma unroll
        for (int j = 0; j < BETA; ++j) {
            kb[j] = ld_stream2(kp + (size_t)j * plane);
            ka[j] = make_double2(key_a(ks[j], r, p, T.logN, q), key_a(ks[j], r, p + 1, T.logN, q));
        }
    }
    for (int e = ch.x; e < ch.x + ch.y; ++e) {
        const int2 tk = tasks[e];
        const IpJob J = jobs[tk.x];
        const IpTerm tm = terms[tk.y];
        const int pp = tm.g == 1 ? p : perm_index(p, tm.g, T.logN);
        const int pb = pp & ~1;
        const bool sw = pp & 1;
        const double *ys = y + (size_t)J.src * BETA * plane + (size_t)r * N;
        double y0[BETA], y1[BETA];
#pragma unroll
        for (int j = 0; j < BETA; ++j) {
            const double2 v = ld2(ys + (size_t)j * plane + pb);
            y0[j] = sw ? v.y : v.x;
            y1[j] = sw ? v.x : v.y;
        }
        double a0x = 0.0, a0y = 0.0, a1x = 0.0, a1y = 0.0;
#pragma unroll
        for (int j = 0; j < BETA; ++j) {
            a0x += mulm(y0[j], kb[j].x, q, qi);
            a0y += mulm(y1[j], kb[j].y, q, qi);
            a1x += mulm(y0[j], ka[j].x, q, qi);
            a1y += mulm(y1[j], ka[j].y, q, qi);
            if (IP_REDUCE_AFTER(j, BETA)) {
                a0x = redm(a0x, q, qi);
                a0y = redm(a0y, q, qi);
                a1x = redm(a1x, q, qi);
                a1y = redm(a1y, q, qi);
            }
        }
        a0x = redm(a0x, q, qi);
        a0y = redm(a0y, q, qi);
        a1x = redm(a1x, q, qi);
        a1y = redm(a1y, q, qi);
        if (tm.mask >= 0) {
            const double2 mv = ld_stream2(masks[tm.mask] + (size_t)r * N + p);
            a0x = mulm(a0x, mv.x, q, qi);
            a0y = mulm(a0y, mv.y, q, qi);
            a1x = mulm(a1x, mv.x, q, qi);
            a1y = mulm(a1y, mv.y, q, qi);
        }
        double *u = U + (size_t)J.slot * 2 * plane + (size_t)r * N + p;
        if (first_round) {
            if (qrow) {
                // unswitched part of the whole job
                double c0x = 0.0, c0y = 0.0, c1x = 0.0, c1y = 0.0;
                for (int t = J.t0; t < J.t0 + J.nt; ++t) {
                    const IpTerm pt = terms[t];
                    if (pt.kind == IP_RELIN) continue;
                    double2 mv = make_double2(1.0, 1.0);
                    if (pt.mask >= 0) mv = ld2(masks[pt.mask] + (size_t)r * N + p);
                    const int qq = pt.g == 1 ? p : perm_index(p, pt.g, T.logN);
                    const bool qs = qq & 1;
                    const double2 cv = ld2(J.c0 + (size_t)r * N + (qq & ~1));
                    double x0 = qs ? cv.y : cv.x, x1 = qs ? cv.x : cv.y;
                    if (pt.mask >= 0) {
                        x0 = mulm(x0, mv.x, q, qi);
                        x1 = mulm(x1, mv.y, q, qi);
                    }
                    c0x = redm(c0x + x0, q, qi);
                    c0y = redm(c0y + x1, q, qi);
                    if (pt.g == 1) {
                        const double2 w = ld2(J.c1 + (size_t)r * N + p);
                        double z0 = w.x, z1 = w.y;
                        if (pt.mask >= 0) {
                            z0 = mulm(z0, mv.x, q, qi);
                            z1 = mulm(z1, mv.y, q, qi);
                        }
                        c1x = redm(c1x + z0, q, qi);
                        c1y = redm(c1y + z1, q, qi);
                    }
                }
                const double P = T.pmod[r];
                a0x = redm(a0x + mulm(c0x, P, q, qi), q, qi);
                a0y = redm(a0y + mulm(c0y, P, q, qi), q, qi);
                a1x = redm(a1x + mulm(c1x, P, q, qi), q, qi);
                a1y = redm(a1y + mulm(c1y, P, q, qi), q, qi);
            }
        } else {
            const double2 u0 = *(const double2 *)u;
            const double2 u1 = *(const double2 *)(u + plane);
            a0x = redm(a0x + u0.x, q, qi);
            a0y = redm(a0y + u0.y, q, qi);
            a1x = redm(a1x + u1.x, q, qi);
            a1y = redm(a1y + u1.y, q, qi);
        }
        *(double2 *)u = make_double2(a0x, a0y);
        *(double2 *)(u + plane) = make_double2(a1x, a1y);
    }
}

// One finished rotation sum at (prime i, position p): a key-switched job's
// output sits in E; otherwise the job adds its terms, each its (c0, c1) or a
// finished rotation E[ks], times the term's mask.
__device__ __forceinline__ void finish_one(const DevTables &T, const FinJob &J, const FinTerm *terms,
                                           const double *E, const double *const *masks, int i, int p, double q,
                                           double qi, double &e0, double &e1) {
    const int N = 1 << T.logN;
    const size_t off = (size_t)i * N;
    const size_t plane = (size_t)T.L * N;
    if (J.ks >= 0) {
        const double *e = E + (size_t)J.ks * 2 * plane + off + p;
        e0 = e[0];
        e1 = e[plane];
        return;
    }
    e0 = 0.0;
    e1 = 0.0;
    for (int t = J.t0; t < J.t0 + J.nt; ++t) {
        const FinTerm ft = terms[t];
        const double *s0 = ft.ks >= 0 ? E + (size_t)ft.ks * 2 * plane : J.c0;
        const double *s1 = ft.ks >= 0 ? s0 + plane : J.c1;
        double x0 = gld(s0)[off + p], x1 = gld(s1)[off + p];
        if (ft.mask >= 0) {
            const double mv = gld(masks[ft.mask])[off + p];
            x0 = mulm(x0, mv, q, qi);
            x1 = mulm(x1, mv, q, qi);
        }
        e0 = redm(e0 + x0, q, qi);
        e1 = redm(e1 + x1, q, qi);
    }
}

// finish_one for the two positions p, p + 1 (p even), 16-byte loads.
__device__ __forceinline__ void finish_two(const DevTables &T, const FinJob &J, const FinTerm *terms,
                                           const double *E, const double *const *masks, int i, int p, double q,
                                           double qi, double2 &e0, double2 &e1) {
    const int N = 1 << T.logN;
    const size_t off = (size_t)i * N + p;
    const size_t plane = (size_t)T.L * N;
    if (J.ks >= 0) {
        const double *e = E + (size_t)J.ks * 2 * plane + off;
        e0 = *(const double2 *)e;
        e1 = *(const double2 *)(e + plane);
        return;
    }
    e0 = make_double2(0.0, 0.0);
    e1 = make_double2(0.0, 0.0);
    for (int t = J.t0; t < J.t0 + J.nt; ++t) {
        const FinTerm ft = terms[t];
        const double *s0 = ft.ks >= 0 ? E + (size_t)ft.ks * 2 * plane : J.c0;
        const double *s1 = ft.ks >= 0 ? s0 + plane : J.c1;
        double2 x0 = ld2(s0 + off), x1 = ld2(s1 + off);
        if (ft.mask >= 0) {
            const double2 mv = ld2(masks[ft.mask] + off);
            x0 = make_double2(mulm(x0.x, mv.x, q, qi), mulm(x0.y, mv.y, q, qi));
            x1 = make_double2(mulm(x1.x, mv.x, q, qi), mulm(x1.y, mv.y, q, qi));
        }
        e0 = make_double2(redm(e0.x + x0.x, q, qi), redm(e0.y + x0.y, q, qi));
        e1 = make_double2(redm(e1.x + x1.x, q, qi), redm(e1.y + x1.y, q, qi));
    }
}

constexpr int FT_P = 64;  // threads along positions per block (two positions each): one wave
constexpr int FT_C = 16;  // pair chunks per block (one per wave), reduced through LDS

// Tensor accumulation: block (128 positions x 16 pair chunks) per (prime i,
// request); each thread takes two adjacent positions and a strided 16th of
// the request's (eps, omega) pairs, then the partial sums are added in LDS.
__global__ void __launch_bounds__(FT_P * FT_C)
k_fin_tensor(DevTables T, const FinJob *jobs, const FinTerm *terms, const double *E, const double *const *masks,
             const int2 *req_pairs, double *const *acc) {
    static_assert(FT_P == 64, "one pair chunk per wave");
    __shared__ double2 part[3][FT_C][FT_P];
    const int N = 1 << T.logN;
    const int p = 2 * (blockIdx.x * FT_P + threadIdx.x);
    // threadIdx.y is the same on every lane of a wave: said so, the job
    // descriptors are scalar loads and the branches on them uniform, instead
    // of a vector load and a wait per field
    const int c = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    const int i = blockIdx.y;
    const int req = blockIdx.z;
    const double q = T.qt[i].x, qi = T.qt[i].y;
    const int2 pr = req_pairs[req];
    double2 a0 = make_double2(0.0, 0.0), a1 = a0, a2 = a0;
    if (p < N) {
        for (int pi = pr.x + c; pi < pr.x + pr.y; pi += FT_C) {
            double2 e0, e1, f0, f1;
            finish_two(T, jobs[2 * pi], terms, E, masks, i, p, q, qi, e0, e1);
            finish_two(T, jobs[2 * pi + 1], terms, E, masks, i, p, q, qi, f0, f1);
            a0.x = redm(a0.x + mulm(e0.x, f0.x, q, qi), q, qi);
            a0.y = redm(a0.y + mulm(e0.y, f0.y, q, qi), q, qi);
            a1.x = redm(a1.x + mulm(e0.x, f1.x, q, qi) + mulm(e1.x, f0.x, q, qi), q, qi);
            a1.y = redm(a1.y + mulm(e0.y, f1.y, q, qi) + mulm(e1.y, f0.y, q, qi), q, qi);
            a2.x = redm(a2.x + mulm(e1.x, f1.x, q, qi), q, qi);
            a2.y = redm(a2.y + mulm(e1.y, f1.y, q, qi), q, qi);
        }
    }
    part[0][c][threadIdx.x] = a0;
    part[1][c][threadIdx.x] = a1;
    part[2][c][threadIdx.x] = a2;
    __syncthreads();
    if (c < 3 && p < N) {
        double sx = 0.0, sy = 0.0;
#pragma unroll
        for (int k = 0; k < FT_C; ++k) {
            sx += part[c][k][threadIdx.x].x;
            sy += part[c][k][threadIdx.x].y;
        }
        st2(acc[req] + (size_t)c * T.L * N + (size_t)i * N + p, make_double2(redm(sx, q, qi), redm(sy, q, qi)));
    }
}

__global__ void __launch_bounds__(EW_THREADS)
k_fin_rotsum(DevTables T, const FinJob *jobs, const FinTerm *terms, const double *E, const double *const *masks,
             double *const *out) {
    const int N = 1 << T.logN;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    const int job = blockIdx.z;
    if (p >= N) return;
    const double q = T.qt[i].x, qi = T.qt[i].y;
    double e0, e1;
    finish_one(T, jobs[job], terms, E, masks, i, p, q, qi, e0, e1);
    auto o = gst(out[job] + (size_t)i * N + p);
    o[0] = e0;
    o[(size_t)T.L * N] = e1;
}

// Group sums of two-component ciphertexts stored one after the other:
// out[g] = sum of in[k] over k in [groups[g].x, groups[g].x + groups[g].y).
// Each thread two adjacent positions of one (component, prime) row.
__global__ void __launch_bounds__(EW_THREADS)
k_sum_cts(DevTables T, const double *in, const int2 *groups, double *const *out) {
    const int N = 1 << T.logN;
    const int p = 2 * (blockIdx.x * blockDim.x + threadIdx.x);
    const int r = blockIdx.y;   // component * L + prime
    const int g = blockIdx.z;
    if (p >= N) return;
    const int i = r % T.L;
    const double q = T.qt[i].x, qi = T.qt[i].y;
    const int2 gr = groups[g];
    const size_t ctw = (size_t)2 * T.L * N;
    double2 a = make_double2(0.0, 0.0);
    for (int k = gr.x; k < gr.x + gr.y; ++k) {
        const double2 v = ld2(in + (size_t)k * ctw + (size_t)r * N + p);
        a.x = redm(a.x + v.x, q, qi);
        a.y = redm(a.y + v.y, q, qi);
    }
    st2(gld(out)[g] + (size_t)r * N + p, a);
}

__global__ void k_copy16(uint4 *dst, const uint4 *src, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

__global__ void k_u64_to_dbl(const uint64_t *in, double *out, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (double)in[i];
}

__global__ void k_dbl_to_u64(const double *in, uint64_t *out, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (uint64_t)in[i];
}

__global__ void k_mul_rows(DevTables T, double *out, const double *a, const double *b, int prime_base,
                           int per) {
    const int N = 1 << T.logN;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (p >= N) return;
    const int pr = prime_base + r % per;
    const double q = T.qt[pr].x, qi = T.qt[pr].y;
    const size_t x = (size_t)r * N + p;
    out[x] = mulm(a[x], b[x], q, qi);
}

__global__ void k_add_rows(DevTables T, double *out, const double *a, const double *b, int prime_base,
                           int per) {
    const int N = 1 << T.logN;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (p >= N) return;
    const int pr = prime_base + r % per;
    const double q = T.qt[pr].x, qi = T.qt[pr].y;
    const size_t x = (size_t)r * N + p;
    out[x] = redm(a[x] + b[x], q, qi);
}

__global__ void k_scale_rows(DevTables T, double *out, const double *a, double c, int per) {
    const int N = 1 << T.logN;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (p >= N) return;
    const int pr = r % per;
    const double q = T.qt[pr].x, qi = T.qt[pr].y;
    const size_t x = (size_t)r * N + p;
    out[x] = mulm(a[x], c, q, qi);
}

__global__ void k_center_rows(DevTables T, double *x, int prime_base, int per) {
    const int N = 1 << T.logN;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (p >= N) return;
    const int pr = prime_base + r % per;
    const size_t ix = (size_t)r * N + p;
    x[ix] = centerm(x[ix], T.qt[pr].x, T.qt[pr].y);
}

// SplitMix64 (Steele, Lea, Flood 2014): the k-th output of the stream that
// starts in state s0 is mix(s0 + (k+1) * golden_gamma).

__global__ void k_sample_uniform(DevTables T, double *out, uint64_t s0, uint64_t first, int prime_base) {
    const int N = 1 << T.logN;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (p >= N) return;
    const uint64_t q = (uint64_t)T.qt[prime_base + r].x;
    const uint64_t v = __umul64hi(sm_draw(s0, first + (uint64_t)r * N + p), q);
    out[(size_t)r * N + p] = (double)v;
}

__constant__ uint64_t c_gauss_cdt[GAUSS_CDT_LEN];

// kind 0: ternary {0, +1, -1} from floor(3 r / 2^64); kind 1: Gaussian by the table.
__global__ void k_sample_small(double *out, uint64_t s0, uint64_t first, int N, int kind) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const uint64_t r = sm_draw(s0, first + i);
    double v;
    if (kind == 0) {
        const uint64_t c = __umul64hi(r, 3ULL);
        v = c == 0 ? 0.0 : (c == 1 ? 1.0 : -1.0);
    } else {
        int c = 0;
        for (int k = 0; k < GAUSS_CDT_LEN; ++k) c += (c_gauss_cdt[k] <= r);
        v = (double)(c - GAUSS_BOUND);
    }
    out[i] = v;
}

__global__ void k_broadcast_rows(const double *x, double *out, int N) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    out[(size_t)blockIdx.y * N + p] = x[p];
}

__global__ void k_axpy_rows(DevTables T, double *out, const double *x, const double *c, const double *y) {
    const int N = 1 << T.logN;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (p >= N) return;
    const double q = T.qt[r].x, qi = T.qt[r].y;
    const size_t ix = (size_t)r * N + p;
    out[ix] = redm(mulm(x[ix], c[r], q, qi) + y[ix], q, qi);
}

// slot s of row 0 <-> exponent 5^s mod 2N <-> natural index (e-1)/2
__global__ void k_scatter_slots(int logN, const double *slots, double *out) {
    const int N = 1 << logN;
    const int S = N >> 1;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    // 5^s mod 2N by square-and-multiply
    unsigned e = 1, b = 5, k = (unsigned)s;
    const unsigned mask = (unsigned)(2 * N - 1);
    while (k) {
        if (k & 1) e = (e * b) & mask;
        b = (b * b) & mask;
        k >>= 1;
    }
    out[brev_bits((int)(e - 1) >> 1, logN)] = slots[s];
    const unsigned e1 = (unsigned)(2 * N) - e;
    out[brev_bits((int)(e1 - 1) >> 1, logN)] = 0.0;
}

__global__ void k_gather_slots(int logN, const double *ev, double *slots) {
    const int N = 1 << logN;
    const int S = N >> 1;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    unsigned e = 1, b = 5, k = (unsigned)s;
    const unsigned mask = (unsigned)(2 * N - 1);
    while (k) {
        if (k & 1) e = (e * b) & mask;
        b = (b * b) & mask;
        k >>= 1;
    }
    slots[s] = ev[brev_bits((int)(e - 1) >> 1, logN)];
}

__global__ void k_automorph_rows(int logN, double *out, const double *in, int g) {
    const int N = 1 << logN;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const size_t off = (size_t)blockIdx.y * N;
    out[off + p] = in[off + perm_index(p, g, logN)];
}

__global__ void k_keygen_combine(DevTables T, double *b, uint64_t a_stream, const double *e, const double *s_,
                                 const double *sp, const double *gadget) {
    const int N = 1 << T.logN;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (p >= N) return;
    const double q = T.qt[r].x, qi = T.qt[r].y;
    const size_t ix = (size_t)r * N + p;
    const double a = key_a(a_stream, r, p, T.logN, q);
    double v = mulm(e[ix], T.t, q, qi) - mulm(a, s_[ix], q, qi);
    v += mulm(sp[ix], gadget[r], q, qi);
    b[ix] = redm(v, q, qi);
}

__global__ void k_enc_noisy(double *out, const double *e, const double *mu, double t, double ti, int N) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    // centered lift of mu (a t-transform output, |mu| < t) plus t e: a small integer
    out[p] = t * e[p] + centerm(mu[p], t, ti);
}

__global__ void k_enc_combine(DevTables T, double *c0, const double *x, const double *a, const double *s_) {
    const int N = 1 << T.logN;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (p >= N) return;
    const double q = T.qt[r].x, qi = T.qt[r].y;
    const size_t ix = (size_t)r * N + p;
    c0[ix] = redm(x[ix] - mulm(a[ix], s_[ix], q, qi), q, qi);
}

__global__ void k_dec_combine(DevTables T, double *v, const double *ct, int comps, const double *s_,
                              const double *s2) {
    const int N = 1 << T.logN;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (p >= N) return;
    const double q = T.qt[r].x, qi = T.qt[r].y;
    const size_t ix = (size_t)r * N + p;
    const size_t plane = (size_t)T.L * N;
    double acc = ct[ix] + mulm(ct[plane + ix], s_[ix], q, qi);
    if (comps > 2) acc += mulm(ct[2 * plane + ix], s2[ix], q, qi);
    v[ix] = redm(acc, q, qi);
}

__global__ void k_scale_small(double *out, const double *x, double c, int N) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < N) out[p] = c * x[p];
}

bool g_cdt_uploaded[64] = {false};

}  // namespace

static dim3 ew_grid(int N, int y, int z = 1) { return dim3((N + EW_THREADS - 1) / EW_THREADS, y, z); }

// A launch whose start and stop timestamps land in ev0 / ev1 (taken by the
// dispatch itself, so they bracket exactly the kernel), or a plain launch.
template <typename... Args, typename F = void (*)(Args...)>
static void launch_timed(F kernel, dim3 grid, dim3 block, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1,
                         Args... args) {
    if (ev0) hipExtLaunchKernelGGL(kernel, grid, block, 0, s, ev0, ev1, 0, args...);
    else hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
}

void ip_launch(const DevTables &T, double *U, const double *y, const double *const *keys, const uint64_t *streams,
               const double *const *masks, const IpJob *jobs, const IpTerm *terms, int njobs, bool transform_pass,
               hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, bool key_reuse) {
    if (njobs <= 0 || njobs > MAX_GRID_Z) {
        // nothing to launch, or the z extent of a launch is limited: split,
        // timed by events around the launches
        if (ev0) (void)hipEventRecord(ev0, s);   // a failed record surfaces when the timing is read
        for (int o = 0; o < njobs; o += MAX_GRID_Z)
            ip_launch(T, U, y, keys, streams, masks, jobs + o, terms, std::min(MAX_GRID_Z, njobs - o),
                      transform_pass, s, nullptr, nullptr, key_reuse);
        if (ev1) (void)hipEventRecord(ev1, s);
        return;
    }
    dim3 grid((T.N / 2 + IP_THREADS - 1) / IP_THREADS, T.nExt, njobs);
    switch (T.beta) {
#define HG_IP_CASE(B)                                                                                        \
    case B:                                                                                                  \
        if (transform_pass && key_reuse)                                                                     \
            launch_timed(k_ip<B, 2>, grid, dim3(IP_THREADS), s, ev0, ev1, T, U, y, keys, streams, masks, jobs, terms); \
        else if (transform_pass)                                                                             \
            launch_timed(k_ip<B, 0>, grid, dim3(IP_THREADS), s, ev0, ev1, T, U, y, keys, streams, masks, jobs, terms); \
        else                                                                                                 \
            launch_timed(k_ip<B, 1>, grid, dim3(IP_THREADS), s, ev0, ev1, T, U, y, keys, streams, masks, jobs, terms); \
        break;
        HG_IP_CASE(1) HG_IP_CASE(2) HG_IP_CASE(3) HG_IP_CASE(4) HG_IP_CASE(5) HG_IP_CASE(6)
        HG_IP_CASE(7) HG_IP_CASE(8) HG_IP_CASE(9) HG_IP_CASE(10) HG_IP_CASE(11) HG_IP_CASE(12)
#undef HG_IP_CASE
        default: break;
    }
}

void ip_one_launch(const DevTables &T, double *U, const double *y, const IpOne &one, hipStream_t s, hipEvent_t ev0,
                   hipEvent_t ev1) {
    bool ok = T.beta >= 1 && T.beta <= IP_ONE_MAX_BETA && one.J.nt >= 1 && one.J.nt <= IP_ONE_MAX_TERMS;
    for (int u = 0; ok && u < one.J.nt; ++u)
        ok = (one.tm[u].kind == IP_PLAIN || one.key) && (one.tm[u].mask < 0 || one.mask[u]);
    if (!ok) throw std::invalid_argument("ip_one_launch: one job of at most two terms, with its key and masks");
    // the terms of a relinearisation (the job's c0, c1 as they are, then the
    // key switch of c2) take the kernel that knows them
    const bool relin = one.J.nt == 2 && one.tm[0].kind == IP_PLAIN && one.tm[0].g == 1 && one.tm[0].mask < 0 &&
                       one.tm[1].kind == IP_RELIN && one.tm[1].g == 1 && one.tm[1].mask < 0;
    dim3 grid((T.N / 2 + IP_THREADS - 1) / IP_THREADS, T.nExt, 1);
    switch (T.beta) {
#define HG_IP1_CASE(B)                                                                       \
    case B:                                                                                  \
        if (relin)                                                                           \
            launch_timed(k_ip_one<B, true>, grid, dim3(IP_THREADS), s, ev0, ev1, T, U, y, one); \
        else                                                                                 \
            launch_timed(k_ip_one<B, false>, grid, dim3(IP_THREADS), s, ev0, ev1, T, U, y, one); \
        break;
        HG_IP1_CASE(1) HG_IP1_CASE(2) HG_IP1_CASE(3) HG_IP1_CASE(4) HG_IP1_CASE(5) HG_IP1_CASE(6)
        HG_IP1_CASE(7) HG_IP1_CASE(8) HG_IP1_CASE(9) HG_IP1_CASE(10) HG_IP1_CASE(11) HG_IP1_CASE(12)
#undef HG_IP1_CASE
        default: break;
    }
}

void ip_keyed_launch(const DevTables &T, double *U, const double *y, const double *const *keys,
                     const uint64_t *streams, const double *const *masks, const IpJob *jobs, const IpTerm *terms,
                     const int2 *chunks, const int2 *tasks, int nchunks, bool first_round, bool transform_pass,
                     hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (nchunks <= 0 || nchunks > MAX_GRID_Z) {
        if (ev0) (void)hipEventRecord(ev0, s);   // a failed record surfaces when the timing is read
        for (int o = 0; o < nchunks; o += MAX_GRID_Z)
            ip_keyed_launch(T, U, y, keys, streams, masks, jobs, terms, chunks + o, tasks,
                            std::min(MAX_GRID_Z, nchunks - o), first_round, transform_pass, s);
        if (ev1) (void)hipEventRecord(ev1, s);
        return;
    }
    dim3 grid((T.N / 2 + IP_THREADS - 1) / IP_THREADS, T.nExt, nchunks);
    const int fr = first_round ? 1 : 0;
    switch (T.beta) {
#define HG_IPK_CASE(B)                                                                                        \
    case B:                                                                                                  \
        if (transform_pass)                                                                                  \
            launch_timed(k_ip_keyed<B, 0>, grid, dim3(IP_THREADS), s, ev0, ev1, T, U, y, keys, streams, masks, jobs, \
                         terms, chunks, tasks, fr);                                                          \
        else                                                                                                 \
            launch_timed(k_ip_keyed<B, 1>, grid, dim3(IP_THREADS), s, ev0, ev1, T, U, y, keys, streams, masks, jobs, \
                         terms, chunks, tasks, fr);                                                          \
        break;
        HG_IPK_CASE(1) HG_IPK_CASE(2) HG_IPK_CASE(3) HG_IPK_CASE(4) HG_IPK_CASE(5) HG_IPK_CASE(6)
        HG_IPK_CASE(7) HG_IPK_CASE(8) HG_IPK_CASE(9) HG_IPK_CASE(10) HG_IPK_CASE(11) HG_IPK_CASE(12)
#undef HG_IPK_CASE
        default: break;
    }
}

void fin_tensor_launch(const DevTables &T, const FinJob *jobs, const FinTerm *terms, const double *E,
                       const double *const *masks, const int2 *req_pairs, double *const *acc, int nreq,
                       hipStream_t s) {
    if (nreq <= 0) return;
    if (nreq > MAX_GRID_Z) {
        for (int o = 0; o < nreq; o += MAX_GRID_Z)
            fin_tensor_launch(T, jobs, terms, E, masks, req_pairs + o, acc + o, std::min(MAX_GRID_Z, nreq - o), s);
        return;
    }
    dim3 grid((T.N + 2 * FT_P - 1) / (2 * FT_P), T.L, nreq);
    hipLaunchKernelGGL(k_fin_tensor, grid, dim3(FT_P, FT_C), 0, s, T, jobs, terms, E, masks, req_pairs, acc);
}

void fin_rotsum_launch(const DevTables &T, const FinJob *jobs, const FinTerm *terms, const double *E,
                       const double *const *masks, double *const *out, int njobs, hipStream_t s) {
    if (njobs <= 0) return;
    if (njobs > MAX_GRID_Z) {
        for (int o = 0; o < njobs; o += MAX_GRID_Z)
            fin_rotsum_launch(T, jobs + o, terms, E, masks, out + o, std::min(MAX_GRID_Z, njobs - o), s);
        return;
    }
    hipLaunchKernelGGL(k_fin_rotsum, ew_grid(T.N, T.L, njobs), dim3(EW_THREADS), 0, s, T, jobs, terms, E, masks,
                       out);
}

void sum_cts_launch(const DevTables &T, const double *in, const int2 *groups, double *const *out, int ngroups,
                    hipStream_t s) {
    if (ngroups <= 0) return;
    if (ngroups > MAX_GRID_Z) {
        for (int o = 0; o < ngroups; o += MAX_GRID_Z)
            sum_cts_launch(T, in, groups + o, out + o, std::min(MAX_GRID_Z, ngroups - o), s);
        return;
    }
    hipLaunchKernelGGL(k_sum_cts, ew_grid(T.N / 2, 2 * T.L, ngroups), dim3(EW_THREADS), 0, s, T, in, groups, out);
}

void copy_from_host(void *dst, const void *src, size_t bytes, hipStream_t s, hipEvent_t done) {
    const size_t n = bytes / 16;
    if (!n) {
        if (done) (void)hipEventRecord(done, s);   // a failed record surfaces at the next wait on it
        return;
    }
    const dim3 grid((unsigned)((n + 255) / 256));
    if (done)   // the dispatch's own completion signal, no separate marker packet
        hipExtLaunchKernelGGL(k_copy16, grid, dim3(256), 0, s, nullptr, done, 0, (uint4 *)dst, (const uint4 *)src, n);
    else
        hipLaunchKernelGGL(k_copy16, grid, dim3(256), 0, s, (uint4 *)dst, (const uint4 *)src, n);
}

void u64_to_dbl(const uint64_t *in, double *out, size_t n, hipStream_t s) {
    if (!n) return;
    hipLaunchKernelGGL(k_u64_to_dbl, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, out, n);
}

void dbl_to_u64(const double *in, uint64_t *out, size_t n, hipStream_t s) {
    if (!n) return;
    hipLaunchKernelGGL(k_dbl_to_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, out, n);
}

void mul_rows(const DevTables &T, double *out, const double *a, const double *b, int rows, int prime_base,
              int per, hipStream_t s) {
    if (rows <= 0) return;
    hipLaunchKernelGGL(k_mul_rows, ew_grid(T.N, rows), dim3(EW_THREADS), 0, s, T, out, a, b, prime_base, per);
}

void add_rows(const DevTables &T, double *out, const double *a, const double *b, int rows, int prime_base,
              int per, hipStream_t s) {
    if (rows <= 0) return;
    hipLaunchKernelGGL(k_add_rows, ew_grid(T.N, rows), dim3(EW_THREADS), 0, s, T, out, a, b, prime_base, per);
}

void scale_rows(const DevTables &T, double *out, const double *a, int rows, int per, double c, hipStream_t s) {
    if (rows <= 0) return;
    hipLaunchKernelGGL(k_scale_rows, ew_grid(T.N, rows), dim3(EW_THREADS), 0, s, T, out, a, c, per);
}

void center_rows(const DevTables &T, double *x, int rows, int prime_base, int per, hipStream_t s) {
    if (rows <= 0) return;
    hipLaunchKernelGGL(k_center_rows, ew_grid(T.N, rows), dim3(EW_THREADS), 0, s, T, x, prime_base, per);
}

void sample_uniform(const DevTables &T, double *out, uint64_t s0, uint64_t first, int rows, int prime_base,
                    hipStream_t s) {
    if (rows <= 0) return;
    hipLaunchKernelGGL(k_sample_uniform, ew_grid(T.N, rows), dim3(EW_THREADS), 0, s, T, out, s0, first, prime_base);
}

void sample_small(double *out, uint64_t s0, uint64_t first, int N, int kind, hipStream_t s) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev >= 0 && dev < 64 && !g_cdt_uploaded[dev]) {
        (void)hipMemcpyToSymbol(HIP_SYMBOL(c_gauss_cdt), GAUSS_CDT, sizeof(GAUSS_CDT));
        g_cdt_uploaded[dev] = true;
    }
    hipLaunchKernelGGL(k_sample_small, dim3((N + 255) / 256), dim3(256), 0, s, out, s0, first, N, kind);
}

void broadcast_rows(const double *x, double *out, int N, int rows, hipStream_t s) {
    if (rows <= 0) return;
    hipLaunchKernelGGL(k_broadcast_rows, ew_grid(N, rows), dim3(EW_THREADS), 0, s, x, out, N);
}

void axpy_rows(const DevTables &T, double *out, const double *x, const double *c, const double *y, int rows,
               hipStream_t s) {
    if (rows <= 0) return;
    hipLaunchKernelGGL(k_axpy_rows, ew_grid(T.N, rows), dim3(EW_THREADS), 0, s, T, out, x, c, y);
}

void scatter_slots(const DevTables &T, const double *slots, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter_slots, dim3((T.N / 2 + 255) / 256), dim3(256), 0, s, T.logN, slots, out);
}

void gather_slots(const DevTables &T, const double *ev, double *slots, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_slots, dim3((T.N / 2 + 255) / 256), dim3(256), 0, s, T.logN, ev, slots);
}

void keygen_combine(const DevTables &T, double *b, uint64_t a_stream, const double *e, const double *s_,
                    const double *sp, const double *gadget, hipStream_t s) {
    hipLaunchKernelGGL(k_keygen_combine, ew_grid(T.N, T.nExt), dim3(EW_THREADS), 0, s, T, b, a_stream, e, s_, sp,
                       gadget);
}

void enc_noisy(const DevTables &T, double *out, const double *e, const double *mu, hipStream_t s) {
    hipLaunchKernelGGL(k_enc_noisy, dim3((T.N + 255) / 256), dim3(256), 0, s, out, e, mu, T.t, T.tinv, T.N);
}

void enc_combine(const DevTables &T, double *c0, const double *noisy_eval, const double *a, const double *s_,
                 hipStream_t s) {
    hipLaunchKernelGGL(k_enc_combine, ew_grid(T.N, T.L), dim3(EW_THREADS), 0, s, T, c0, noisy_eval, a, s_);
}

void dec_combine(const DevTables &T, double *v, const double *ct, int comps, const double *s_, const double *s2,
                 hipStream_t s) {
    hipLaunchKernelGGL(k_dec_combine, ew_grid(T.N, T.L), dim3(EW_THREADS), 0, s, T, v, ct, comps, s_, s2);
}

void scale_small(double *out, const double *x, double c, int N, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_small, dim3((N + 255) / 256), dim3(256), 0, s, out, x, c, N);
}

void automorph_rows(const DevTables &T, double *out, const double *in, int rows, int g, hipStream_t s) {
    if (rows <= 0) return;
    hipLaunchKernelGGL(k_automorph_rows, ew_grid(T.N, rows), dim3(EW_THREADS), 0, s, T.logN, out, in, g);
}

}  // namespace hg
