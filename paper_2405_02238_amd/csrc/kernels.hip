// HIP kernels for gfx950: negacyclic transforms, digit lifting, key-switch
// inner products, the division by P, tensor accumulation, sampling.
#include "kernels.h"

#include "arith.h"
#include "gauss_cdt.h"

namespace hg {

namespace {

constexpr int NTT_THREADS_MAX = 512;

__device__ __forceinline__ int brev_bits(int x, int bits) {
    return (int)(__brev((unsigned)x) >> (32 - bits));
}

// Evaluation-form automorphism X -> X^g: position p holds the value at
// psi^(2 brv(p) + 1).  The permuted polynomial's value there is the source
// value at psi^((2 brv(p) + 1) g): natural index ((2i+1) g mod 2N - 1) / 2.
__device__ __forceinline__ int perm_index(int p, int g, int logN) {
    int i = brev_bits(p, logN);
    int twoN = 2 << logN;
    int e = (int)(((long long)(2 * i + 1) * g) & (twoN - 1));
    return brev_bits((e - 1) >> 1, logN);
}

// One workgroup transforms one row held in LDS.  Rounds of up to three
// radix-2 stages run in registers on groups of eight elements; LDS carries
// the data between rounds.
template <int LOAD>
__global__ void __launch_bounds__(NTT_THREADS_MAX)
k_ntt_fwd(DevTables T, NttArgs a) {
    extern __shared__ double sh[];
    const int row = blockIdx.x;
    const int logN = T.logN;
    const int N = 1 << logN;
    int prime;
    double *out;
    if (LOAD == LOAD_MODUP) {
        const int r = row % T.nExt;
        const int j = (row / T.nExt) % T.beta;
        const int src = row / (T.nExt * T.beta);
        prime = r;
        out = a.out + (size_t)row * N;
        const double *c = a.in + (size_t)src * a.in_stride;
        const int d0 = j * T.alpha;
        const int d1 = min(d0 + T.alpha, T.L);
        const double qr = T.qt[r].x, qir = T.qt[r].y;
        if (r >= d0 && r < d1) {
            for (int i = threadIdx.x; i < N; i += blockDim.x) sh[i] = c[(size_t)r * N + i];
        } else if (d1 - d0 == 1) {
            // one-prime digit: the centered residue itself is the lift
            const double qd = T.qt[d0].x, qid = T.qt[d0].y;
            for (int i = threadIdx.x; i < N; i += blockDim.x)
                sh[i] = centerm(c[(size_t)d0 * N + i], qd, qid);
        } else {
            for (int i = threadIdx.x; i < N; i += blockDim.x) {
                double acc = 0.0;
                for (int s = d0; s < d1; ++s) {
                    const double qs = T.qt[s].x, qis = T.qt[s].y;
                    double ct = centerm(mulm(c[(size_t)s * N + i], T.mu_invhat[s], qs, qis), qs, qis);
                    acc += mulm(ct, T.mu_hat[s * T.nExt + r], qr, qir);
                }
                sh[i] = redm(acc, qr, qir);
            }
        }
    } else if (LOAD == LOAD_DELTA) {
        const int i_q = row % T.L;
        const int slot = row / T.L;
        prime = i_q;
        out = a.out + (size_t)row * N;
        const double *rk = a.in + (size_t)slot * a.in_stride;
        const double qr = T.qt[i_q].x, qir = T.qt[i_q].y;
        for (int i = threadIdx.x; i < N; i += blockDim.x) {
            double acc = 0.0;
            for (int k = 0; k < T.alpha; ++k)
                acc += mulm(rk[(size_t)k * N + i], T.md_hat[k * T.L + i_q], qr, qir);
            sh[i] = redm(acc, qr, qir);
        }
    } else {
        const int g = row / a.per, rr = row % a.per;
        prime = a.prime_base + rr;
        out = a.out + (size_t)g * a.out_stride + (size_t)rr * N;
        const double *in = a.in + (size_t)g * a.in_stride + a.in_offset + (size_t)rr * N;
        for (int i = threadIdx.x; i < N; i += blockDim.x) sh[i] = in[i];
    }
    __syncthreads();
    const double q = T.qt[prime].x, qi = T.qt[prime].y;
    const double *tw = T.twf + (size_t)prime * N;
    for (int s0 = 0; s0 < logN;) {
        const int k = min(3, logN - s0);
        const int lts = logN - s0 - k;           // log2 of the smallest half-size ts
        const int ts = 1 << lts;
        const int ngroups = N >> k;
        for (int grp = threadIdx.x; grp < ngroups; grp += blockDim.x) {
            const int low = grp & (ts - 1);
            const int blk = grp >> lts;
            const int base = (blk << (lts + k)) + low;
            double x[8];
#pragma unroll
            for (int b = 0; b < 8; ++b)
                if (b < (1 << k)) x[b] = sh[base + b * ts];
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                if (u >= k) break;
                const int m = 1 << (s0 + u);
                const int half = 1 << (k - 1 - u);
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    if (b >= (1 << k) || (b & half)) continue;
                    const double w = tw[m + (blk << u) + (b >> (k - u))];
                    const double t = mulm(x[b + half], w, q, qi);
                    const double X = x[b];
                    x[b] = redm(X + t, q, qi);
                    x[b + half] = redm(X - t, q, qi);
                }
            }
#pragma unroll
            for (int b = 0; b < 8; ++b)
                if (b < (1 << k)) sh[base + b * ts] = x[b];
        }
        __syncthreads();
        s0 += k;
    }
    for (int i = threadIdx.x; i < N; i += blockDim.x) out[i] = sh[i];
}

template <int STORE>
__global__ void __launch_bounds__(NTT_THREADS_MAX)
k_ntt_inv(DevTables T, NttArgs a) {
    extern __shared__ double sh[];
    const int row = blockIdx.x;
    const int logN = T.logN;
    const int N = 1 << logN;
    const int g = row / a.per, rr = row % a.per;
    const int prime = a.prime_base + rr;
    double *out = a.out + (size_t)g * a.out_stride + (size_t)rr * N;
    const double *in = a.in + (size_t)g * a.in_stride + a.in_offset + (size_t)rr * N;
    for (int i = threadIdx.x; i < N; i += blockDim.x) sh[i] = in[i];
    __syncthreads();
    const double q = T.qt[prime].x, qi = T.qt[prime].y;
    const double *tw = T.twi + (size_t)prime * N;
    for (int shi = logN - 1; shi >= 0;) {
        const int k = min(3, shi + 1);
        const int lts = logN - shi - 1;          // first stage of the round has half-size ts
        const int ts = 1 << lts;
        const int ngroups = N >> k;
        for (int grp = threadIdx.x; grp < ngroups; grp += blockDim.x) {
            const int low = grp & (ts - 1);
            const int blk = grp >> lts;
            const int base = (blk << (lts + k)) + low;
            double x[8];
#pragma unroll
            for (int b = 0; b < 8; ++b)
                if (b < (1 << k)) x[b] = sh[base + b * ts];
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                if (u >= k) break;
                const int h = N >> (lts + u + 1);     // N / (2 t), t = ts << u
                const int d = 1 << u;
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    if (b >= (1 << k) || (b & d)) continue;
                    const double w = tw[h + (blk << (k - u - 1)) + (b >> (u + 1))];
                    const double X = x[b], Y = x[b + d];
                    x[b] = redm(X + Y, q, qi);
                    x[b + d] = mulm(X - Y, w, q, qi);
                }
            }
#pragma unroll
            for (int b = 0; b < 8; ++b)
                if (b < (1 << k)) sh[base + b * ts] = x[b];
        }
        __syncthreads();
        shi -= k;
    }
    if (STORE == STORE_MDR) {
        const double c = T.md_coef[rr];
        for (int i = threadIdx.x; i < N; i += blockDim.x) out[i] = centerm(mulm(sh[i], c, q, qi), q, qi);
    } else {
        const double c = T.ninv[prime];
        for (int i = threadIdx.x; i < N; i += blockDim.x) {
            double v = mulm(sh[i], c, q, qi);
            if (STORE == STORE_CANON) v = canonm(centerm(v, q, qi), q);
            out[i] = v;
        }
    }
}

constexpr int EW_THREADS = 256;

// Key-switching inner products with the automorphism folded into the gather
// of the hoisted digits.  grid: (N / 256, nExt, jobs).
__global__ void __launch_bounds__(EW_THREADS)
k_ip(DevTables T, double *U, const double *y, const double *const *keys, const double *const *masks,
     const int2 *jobs, const IpTerm *terms) {
    const int N = 1 << T.logN;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    const int job = blockIdx.z;
    if (p >= N) return;
    const double q = T.qt[r].x, qi = T.qt[r].y;
    const size_t plane = (size_t)T.nExt * N;           // one digit (or component) of all primes
    const int2 jt = jobs[job];
    double acc0 = 0.0, acc1 = 0.0;
    for (int tix = jt.x; tix < jt.x + jt.y; ++tix) {
        const IpTerm tm = terms[tix];
        const int pp = tm.g == 1 ? p : perm_index(p, tm.g, T.logN);
        const double *ys = y + (size_t)tm.src * T.beta * plane + (size_t)r * N + pp;
        const double *kb = keys[tm.key] + (size_t)r * N + p;
        double s0 = 0.0, s1 = 0.0;
        for (int j = 0; j < T.beta; ++j) {
            const double yv = ys[(size_t)j * plane];
            s0 += mulm(yv, kb[(size_t)(2 * j) * plane], q, qi);
            s1 += mulm(yv, kb[(size_t)(2 * j + 1) * plane], q, qi);
        }
        s0 = redm(s0, q, qi);
        s1 = redm(s1, q, qi);
        if (tm.mask >= 0) {
            const double mv = masks[tm.mask][(size_t)r * N + p];
            s0 = mulm(s0, mv, q, qi);
            s1 = mulm(s1, mv, q, qi);
        }
        acc0 = redm(acc0 + s0, q, qi);
        acc1 = redm(acc1 + s1, q, qi);
    }
    double *u = U + (size_t)job * 2 * plane + (size_t)r * N + p;
    u[0] = acc0;
    u[plane] = acc1;
}

// One finished rotation sum at (prime i, position p).
__device__ __forceinline__ void finish_one(const DevTables &T, const FinJob &J, const FinTerm *terms,
                                           const double *U, const double *delta,
                                           const double *const *masks, int i, int p, double q, double qi,
                                           double &e0, double &e1) {
    const int N = 1 << T.logN;
    const size_t off = (size_t)i * N;
    e0 = 0.0;
    e1 = 0.0;
    for (int t = J.t0; t < J.t0 + J.nt; ++t) {
        const FinTerm ft = terms[t];
        if (ft.g == 1) {
            double x0 = J.c0[off + p], x1 = J.c1[off + p];
            if (ft.mask >= 0) {
                const double mv = masks[ft.mask][off + p];
                x0 = mulm(x0, mv, q, qi);
                x1 = mulm(x1, mv, q, qi);
            }
            e0 = redm(e0 + x0, q, qi);
            e1 = redm(e1 + x1, q, qi);
        } else {
            double x0 = J.c0[off + perm_index(p, ft.g, T.logN)];
            if (ft.mask >= 0) x0 = mulm(x0, masks[ft.mask][off + p], q, qi);
            e0 = redm(e0 + x0, q, qi);
        }
    }
    if (J.ks >= 0) {
        const size_t uplane = (size_t)T.nExt * N;
        const size_t dplane = (size_t)T.L * N;
        const double *u = U + (size_t)J.ks * 2 * uplane + off + p;
        const double *dl = delta + (size_t)J.ks * 2 * dplane + off + p;
        const double pinv = T.pinv[i];
        e0 = redm(e0 + mulm(u[0] - dl[0], pinv, q, qi), q, qi);
        e1 = redm(e1 + mulm(u[uplane] - dl[dplane], pinv, q, qi), q, qi);
    }
}

__global__ void __launch_bounds__(EW_THREADS)
k_fin_tensor(DevTables T, const FinJob *jobs, const FinTerm *terms, const double *U, const double *delta,
             const double *const *masks, const int2 *req_pairs, double *const *acc) {
    const int N = 1 << T.logN;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    const int req = blockIdx.z;
    if (p >= N) return;
    const double q = T.qt[i].x, qi = T.qt[i].y;
    const int2 pr = req_pairs[req];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int pi = pr.x; pi < pr.x + pr.y; ++pi) {
        double e0, e1, f0, f1;
        finish_one(T, jobs[2 * pi], terms, U, delta, masks, i, p, q, qi, e0, e1);
        finish_one(T, jobs[2 * pi + 1], terms, U, delta, masks, i, p, q, qi, f0, f1);
        a0 = redm(a0 + mulm(e0, f0, q, qi), q, qi);
        a1 = redm(a1 + mulm(e0, f1, q, qi) + mulm(e1, f0, q, qi), q, qi);
        a2 = redm(a2 + mulm(e1, f1, q, qi), q, qi);
    }
    const size_t plane = (size_t)T.L * N;
    double *o = acc[req] + (size_t)i * N + p;
    o[0] = a0;
    o[plane] = a1;
    o[2 * plane] = a2;
}

__global__ void __launch_bounds__(EW_THREADS)
k_fin_rotsum(DevTables T, const FinJob *jobs, const FinTerm *terms, const double *U, const double *delta,
             const double *const *masks, double *const *out) {
    const int N = 1 << T.logN;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    const int job = blockIdx.z;
    if (p >= N) return;
    const double q = T.qt[i].x, qi = T.qt[i].y;
    double e0, e1;
    finish_one(T, jobs[job], terms, U, delta, masks, i, p, q, qi, e0, e1);
    double *o = out[job] + (size_t)i * N + p;
    o[0] = e0;
    o[(size_t)T.L * N] = e1;
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
__device__ __forceinline__ uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t sm_draw(uint64_t s0, uint64_t k) {
    return sm_mix(s0 + (k + 1) * 0x9E3779B97F4A7C15ULL);
}

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

__global__ void k_keygen_combine(DevTables T, double *b, const double *a, const double *e, const double *s_,
                                 const double *sp, const double *gadget) {
    const int N = 1 << T.logN;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (p >= N) return;
    const double q = T.qt[r].x, qi = T.qt[r].y;
    const size_t ix = (size_t)r * N + p;
    double v = mulm(e[ix], T.t, q, qi) - mulm(a[ix], s_[ix], q, qi);
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

void kernels_init() {
    const int lds = 160 * 1024;
    (void)hipFuncSetAttribute((const void *)k_ntt_fwd<LOAD_PLAIN>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void *)k_ntt_fwd<LOAD_MODUP>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void *)k_ntt_fwd<LOAD_DELTA>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void *)k_ntt_inv<STORE_PLAIN>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void *)k_ntt_inv<STORE_MDR>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void *)k_ntt_inv<STORE_CANON>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

static int ntt_threads(int N) { return min(N / 8, NTT_THREADS_MAX) < 64 ? 64 : min(N / 8, NTT_THREADS_MAX); }

void ntt_fwd(const DevTables &T, NttLoad mode, const NttArgs &a, hipStream_t s) {
    if (a.rows <= 0) return;
    const int N = T.N;
    const size_t lds = (size_t)N * sizeof(double);
    dim3 grid(a.rows), block(ntt_threads(N));
    switch (mode) {
        case LOAD_MODUP: hipLaunchKernelGGL(k_ntt_fwd<LOAD_MODUP>, grid, block, lds, s, T, a); break;
        case LOAD_DELTA: hipLaunchKernelGGL(k_ntt_fwd<LOAD_DELTA>, grid, block, lds, s, T, a); break;
        default: hipLaunchKernelGGL(k_ntt_fwd<LOAD_PLAIN>, grid, block, lds, s, T, a); break;
    }
}

void ntt_inv(const DevTables &T, NttStore mode, const NttArgs &a, hipStream_t s) {
    if (a.rows <= 0) return;
    const int N = T.N;
    const size_t lds = (size_t)N * sizeof(double);
    dim3 grid(a.rows), block(ntt_threads(N));
    switch (mode) {
        case STORE_MDR: hipLaunchKernelGGL(k_ntt_inv<STORE_MDR>, grid, block, lds, s, T, a); break;
        case STORE_CANON: hipLaunchKernelGGL(k_ntt_inv<STORE_CANON>, grid, block, lds, s, T, a); break;
        default: hipLaunchKernelGGL(k_ntt_inv<STORE_PLAIN>, grid, block, lds, s, T, a); break;
    }
}

static dim3 ew_grid(int N, int y, int z = 1) { return dim3((N + EW_THREADS - 1) / EW_THREADS, y, z); }

void ip_launch(const DevTables &T, double *U, const double *y, const double *const *keys,
               const double *const *masks, const int2 *jobs, const IpTerm *terms, int njobs, hipStream_t s) {
    if (njobs <= 0) return;
    hipLaunchKernelGGL(k_ip, ew_grid(T.N, T.nExt, njobs), dim3(EW_THREADS), 0, s, T, U, y, keys, masks, jobs, terms);
}

void fin_tensor_launch(const DevTables &T, const FinJob *jobs, const FinTerm *terms, const double *U,
                       const double *delta, const double *const *masks, const int2 *req_pairs,
                       double *const *acc, int nreq, hipStream_t s) {
    if (nreq <= 0) return;
    hipLaunchKernelGGL(k_fin_tensor, ew_grid(T.N, T.L, nreq), dim3(EW_THREADS), 0, s, T, jobs, terms, U, delta,
                       masks, req_pairs, acc);
}

void fin_rotsum_launch(const DevTables &T, const FinJob *jobs, const FinTerm *terms, const double *U,
                       const double *delta, const double *const *masks, double *const *out, int njobs,
                       hipStream_t s) {
    if (njobs <= 0) return;
    hipLaunchKernelGGL(k_fin_rotsum, ew_grid(T.N, T.L, njobs), dim3(EW_THREADS), 0, s, T, jobs, terms, U, delta,
                       masks, out);
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

void keygen_combine(const DevTables &T, double *b, const double *a, const double *e, const double *s_,
                    const double *sp, const double *gadget, hipStream_t s) {
    hipLaunchKernelGGL(k_keygen_combine, ew_grid(T.N, T.nExt), dim3(EW_THREADS), 0, s, T, b, a, e, s_, sp, gadget);
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
