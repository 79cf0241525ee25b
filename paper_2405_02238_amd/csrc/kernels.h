// Device data layout and kernel launchers.
//
// Layout in HBM (all doubles holding exact integers, see arith.h):
//  - a polynomial over a set of primes is `rows x N`, one row per prime,
//    limb-major (all N residues of a prime contiguous), 256-byte aligned;
//  - a ciphertext is components x L x N (c0 rows, then c1 rows), kept in the
//    evaluation form produced by k_ntt_fwd (bit-reversed order);
//  - the extended basis orders its rows q_0..q_{L-1}, p_0..p_{alpha-1}; the
//    plaintext modulus t has prime index L + alpha in the tables;
//  - hoisted digits of a source polynomial: beta x (L+alpha) x N;
//  - a switching key: beta x 2 x (L+alpha) x N (b_j rows, then a_j rows).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace hg {

// Per-context tables on the device.
struct DevTables {
    int N = 0, logN = 0, L = 0, alpha = 0, beta = 0, nExt = 0;
    double2 *qt = nullptr;      // [nExt + 1]: (q, fl(1/q)); index nExt is t
    double *twf = nullptr;      // [nExt + 1][N]: psi^brv(i), centered
    double *twi = nullptr;      // [nExt + 1][N]: psi^-brv(i), centered
    double *ninv = nullptr;     // [nExt + 1]: N^-1, centered
    double *mu_invhat = nullptr;  // [L]: ((D_j/q_i) mod q_i)^-1 for q_i in digit j
    double *mu_hat = nullptr;     // [L][nExt]: (D_j/q_i) mod prime r
    double *md_coef = nullptr;    // [alpha]: N^-1 t^-1 (P/p_k)^-1 mod p_k, centered
    double *md_hat = nullptr;     // [alpha][L]: t (P/p_k) mod q_i
    double *pinv = nullptr;       // [L]: P^-1 mod q_i, centered
    double *pmod = nullptr;       // [L]: P mod q_i, centered
    double t = 0.0, tinv = 0.0;   // plaintext modulus and fl(1/t), by value
    // Launch-shape knobs of the context's transforms (host side, bit-neutral):
    int row_rk = 0;       // radix exponent of 4096- and 8192-point rows (3, 4; 0: built-in)
    int half_rows = 128;  // fused chains of at most this many rows split their forward transforms in halves
    int split_rows = 0;   // transforms of fewer rows split each row over N/1024 workgroups (0: only N > 16384)
    int xcd_rows = 1;     // 1: one-workgroup forward rows assigned to XCDs in contiguous blocks (0: by index)
};

// Terms of an inner-product job.  A job computes, over the extended basis,
//   U = P * sum_plain mask (.) phi_g(c0)   [+ P * mask (.) c1 on component 1 when g = 1]
//     + sum_rot   mask (.) KS_g(src)        (inner product of the permuted hoisted digits)
//     + KS_relin(src)
// so that the division by P of U yields the finished rotation sum directly.
enum IpKind { IP_ROT = 0, IP_PLAIN = 1, IP_RELIN = 2 };

struct IpTerm {
    int g;      // Galois element (1 = no permutation)
    int mask;   // index into the mask pointer table, -1 = none
    int key;    // index into the key pointer table, -1 = none (IP_PLAIN)
    int kind;   // IpKind
};

struct IpJob {
    const double *c0;   // L x N, evaluation form (source of the unswitched part)
    const double *c1;
    int src;            // hoisted digit set for the key-switched terms
    int t0, nt;         // terms [t0, t0 + nt)
    int slot;           // output slot of U (the job's index in its pass; the
                        // launch order of the jobs may differ)
};

// One term of a finishing job: the job's own (c0, c1), or (ks >= 0) the
// finished rotation E[ks] of a key-switched job, times the mask.  The
// second form composes a transform in the primitive order of the diagonal
// method: every rotation divided by P on its own, its mask applied after.
struct FinTerm {
    int g;      // must be 1
    int mask;   // -1 = none
    int ks;     // -1: the job's c0, c1; >= 0: the key-switch slot E[ks]
};

struct FinJob {
    const double *c0;   // L x N, evaluation form
    const double *c1;
    int ks;             // key-switch slot: the finished output is E[ks]; -1: use the terms
    int t0, nt;         // terms [t0, t0 + nt)
};

enum NttLoad { LOAD_PLAIN = 0, LOAD_MODUP = 1, LOAD_DELTA = 2, LOAD_DELTA_H = 3 };
enum NttStore { STORE_PLAIN = 0, STORE_MDR = 1, STORE_CANON = 2, STORE_MDR_H = 3 };

struct NttArgs {
    double *out = nullptr;
    const double *in = nullptr;
    int rows = 0;
    int per = 1;               // rows per group
    int prime_base = 0;
    long long out_stride = 0;  // elements between groups
    long long in_stride = 0;
    long long in_offset = 0;
    const double *const *in_tab = nullptr;  // LOAD_PLAIN / inverse: per-group source pointers (device)
    const double *aux = nullptr;            // LOAD_DELTA: U (the un-divided sums), slot stride nExt*N
    // STORE_MDR with halves: two workgroups per row each run the first logN - 1
    // stages on one input half and store them unscaled; the matching
    // LOAD_DELTA (halves) applies the last stage and the centering while it
    // loads (one special prime only; see ntt_halves_ok)
    int halves = 0;
};

// Forward transform of `rows` rows (natural order in, bit-reversed out).
//  LOAD_PLAIN: row r = group r/per, prime prime_base + r%per, in place allowed.
//  LOAD_MODUP: rows are (src, digit j, prime r) over nsrc sources; `in` holds
//              coefficient-form L-row sources with stride in_stride; output
//              row index (src*beta + j)*nExt + r, contiguous.
//  LOAD_DELTA: rows are (slot, i) with i over the L ciphertext primes; `in`
//              holds alpha rows of centered r_k per slot (stride in_stride);
//              the transform of delta_i is subtracted from U_i (aux) and the
//              difference multiplied by P^-1: output E_i = (U_i - delta_i)/P,
//              contiguous slot*L + i.
// ev0 / ev1 (optional) receive the start and end of the launch (of the two
// launches of a split transform, bracketed by stream markers).
void ntt_fwd(const DevTables &T, NttLoad mode, const NttArgs &a, hipStream_t s, hipEvent_t ev0 = nullptr,
             hipEvent_t ev1 = nullptr);

// Inverse transform (bit-reversed in, natural out).
//  STORE_PLAIN: times N^-1.
//  STORE_MDR:   row = (slot, k), prime L + k; output centered
//               r_k = [u_{p_k} N^-1 t^-1 (P/p_k)^-1]_{p_k}, exact.
//  STORE_CANON: times N^-1, canonical residue in [0, q).
void ntt_inv(const DevTables &T, NttStore mode, const NttArgs &a, hipStream_t s);

// Fused chains for one-prime digits (alpha = 1, N <= 16384), one workgroup
// per output row, for passes with few rows:
//  hoist_fused:   y[src][j][r] = NTT_r(center(INTT_j(c1[src] row j)))
//  moddown_fused: E[slot][i] = (U_i - NTT_i(t (P/p) center(INTT_p(U_p) ...))) P^-1
bool fused_ok(const DevTables &T);
void hoist_fused(const DevTables &T, double *y, const double *const *srcs, int nsrc, hipStream_t s);

// hoist_fused with its sources by value and a copy out of pinned host memory
// (a call's descriptor tables, needed by the launches after it) done by extra
// workgroups of the same launch: n16 16-byte words from copy_src (device
// address of pinned memory) to copy_dst.  `done` (optional) is recorded by
// the launch's own completion.  At most HOIST_MAX_SRC sources and
// HOIST_MAX_COPY words (hoist_copy_ok).
constexpr int HOIST_MAX_SRC = 8;
constexpr size_t HOIST_MAX_COPY = (size_t)1 << 16;
struct HoistSrc {
    const double *p[HOIST_MAX_SRC];
    const uint4 *copy_src;
    uint4 *copy_dst;
    unsigned long long copy_n;
    int copy_wgs;
};
bool hoist_copy_ok(int nsrc, size_t copy_bytes);
void hoist_fused_copy(const DevTables &T, double *y, const HoistSrc &a, int nsrc, hipStream_t s, hipEvent_t done);
// hoist_fused with its sources a.p[0 .. nsrc) by value and no copy (the
// copy fields are ignored): the row loads start without a table read first.
void hoist_fused_v(const DevTables &T, double *y, const HoistSrc &a, int nsrc, hipStream_t s);
void moddown_fused(const DevTables &T, double *E, const double *U, int nslots, hipStream_t s,
                   double *const *outs = nullptr);

// Knob values of DevTables::row_rk / half_rows / split_rows:
//  - split_rows: transforms of fewer rows than this are split into a column
//    pass and a block pass of 1024-element workgroups (spreading each row
//    over N/1024 CUs); rows longer than 16384 always use the split form;
//  - row_rk: radix exponent of the 4096- and 8192-point row transforms,
//    3 (radix 8, the built-in choice) or 4 (radix 16); other lengths have
//    one radix;
//  - half_rows: fused chains (hoist_fused, moddown_fused) of at most this
//    many rows run two workgroups per row, each finishing half of the forward
//    transform after applying its first stage (the inverse is done by both);
//    0: off, default 128 (one workgroup per CU at most).
// Results are the same for every setting.  Returns the row_rk of a radix
// (0, 8 or 16); throws std::invalid_argument for other values.
int ntt_radix_rk(int radix);
// Whether a division by P whose inverse has `rows` rows may use the halves
// form of STORE_MDR / LOAD_DELTA (one special prime, one-workgroup rows, at
// most half_rows rows, no split-row transforms).
bool ntt_halves_ok(const DevTables &T, int rows);

// Inner products: U[slot][c][r][p] = sum over the job's key-switched terms of
// mask[r][p] * sum_j key[j][c][r][p] * y[src][j][r][perm_g(p)], plus P times
// the unswitched part on the ciphertext primes (see IpTerm).
// ev0 / ev1 (optional) receive the start and end of the launch.  Keys and
// masks are read with non-temporal loads (each word once per launch), or,
// with key_reuse (the launch's terms share keys, jobs in key order),
// through the caches, so that jobs started side by side find them there.
void ip_launch(const DevTables &T, double *U, const double *y, const double *const *keys, const uint64_t *streams,
               const double *const *masks, const IpJob *jobs, const IpTerm *terms, int njobs,
               bool transform_pass, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
               bool key_reuse = false);

// A launch of one job of at most two terms whose key-switched terms share
// one key (a relinearisation: the unswitched term and the key switch of
// c2; a single rotation), everything the kernel would look up in the pass's
// tables given by value, so that its loads of keys, digits and masks start
// without three dependent table reads first.  J.t0 is not used.
constexpr int IP_ONE_MAX_BETA = 12;
constexpr int IP_ONE_MAX_TERMS = 2;
struct IpOne {
    IpJob J;
    IpTerm tm[IP_ONE_MAX_TERMS];
    const double *mask[IP_ONE_MAX_TERMS];   // each term's mask (null: none)
    const double *key;                      // b half of the key (null: no key-switched term)
    uint64_t st[IP_ONE_MAX_BETA];           // a-half streams of that key, one per digit
};
void ip_one_launch(const DevTables &T, double *U, const double *y, const IpOne &one, hipStream_t s,
                   hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// Key-stationary variant, one launch per round of key-switched terms:
// tasks[i] = (job, term); chunks[c] = (first task, count), all tasks of a
// chunk share one key and no job appears twice in a round.  The first round
// writes U (adding each job's unswitched part), later rounds add to it.
void ip_keyed_launch(const DevTables &T, double *U, const double *y, const double *const *keys,
                     const uint64_t *streams, const double *const *masks, const IpJob *jobs, const IpTerm *terms,
                     const int2 *chunks, const int2 *tasks, int nchunks, bool first_round, bool transform_pass,
                     hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// Tensor-accumulate: per request, sum over its (eps job, omega job) pairs of
// the tensor product of the two finished transforms (E slots or plain terms).
void fin_tensor_launch(const DevTables &T, const FinJob *jobs, const FinTerm *terms, const double *E,
                       const double *const *masks, const int2 *req_pairs, double *const *acc, int nreq,
                       hipStream_t s);

// Finished rotation sums written as ciphertexts: out[job] = E[ks] (or the plain terms).
void fin_rotsum_launch(const DevTables &T, const FinJob *jobs, const FinTerm *terms, const double *E,
                       const double *const *masks, double *const *out, int njobs, hipStream_t s);

// Group sums of ciphertexts (2 x L x N each, evaluation form) stored one
// after the other from `in`: out[g] = sum of ciphertexts groups[g].x ..
// groups[g].x + groups[g].y - 1 (device tables `groups` and `out`).
void sum_cts_launch(const DevTables &T, const double *in, const int2 *groups, double *const *out, int ngroups,
                    hipStream_t s);

// Allow the transform kernels the full LDS of a CDNA4 workgroup (call once
// per device before the first transform with N > 4096).
void kernels_init();

// ---- utilities ----
// Copy `bytes` (a multiple of 16) from device-mapped pinned host memory;
// `done` (optional) is recorded by the copy's own completion.
void copy_from_host(void *dst, const void *src_host_mapped, size_t bytes, hipStream_t s, hipEvent_t done = nullptr);
void u64_to_dbl(const uint64_t *in, double *out, size_t n, hipStream_t s);
void dbl_to_u64(const double *in, uint64_t *out, size_t n, hipStream_t s);
void mul_rows(const DevTables &T, double *out, const double *a, const double *b, int rows,
              int prime_base, int per, hipStream_t s);
void add_rows(const DevTables &T, double *out, const double *a, const double *b, int rows,
              int prime_base, int per, hipStream_t s);
// out = c * a row by row; row r is over prime r % per (|c| below every prime).
void scale_rows(const DevTables &T, double *out, const double *a, int rows, int per, double c, hipStream_t s);

// Sampling (counter-based SplitMix64 streams): rows x N uniform residues
// (draw first + r*N + i), N ternary or Gaussian integers (draw first + i).
void sample_uniform(const DevTables &T, double *out, uint64_t s0, uint64_t first, int rows,
                    int prime_base, hipStream_t s);
void sample_small(double *out, uint64_t s0, uint64_t first, int N, int kind, hipStream_t s);

// Reduce a small signed integer polynomial (N doubles) into rows x N.
void broadcast_rows(const double *x, double *out, int N, int rows, hipStream_t s);
// out[r] = x[r] * c[r] + y[r] for a per-row constant (used by key generation)
void axpy_rows(const DevTables &T, double *out, const double *x, const double *c, const double *y,
               int rows, hipStream_t s);
// Scatter row-0 slot values (S doubles in [0,t)) to the evaluation positions
// of the t-transform (bit-reversed order); row 1 positions get 0.
void scatter_slots(const DevTables &T, const double *slots, double *out, hipStream_t s);
// Gather row-0 slots from a t-transform evaluation vector.
void gather_slots(const DevTables &T, const double *ev, double *slots, hipStream_t s);
// Automorphism in evaluation form: out[p] = in[perm_g(p)] for rows.
void automorph_rows(const DevTables &T, double *out, const double *in, int rows, int g, hipStream_t s);
// Centered canonical representative per row (prime_base + r % per).
void center_rows(const DevTables &T, double *x, int rows, int prime_base, int per, hipStream_t s);
// Switching-key digit, evaluation form over the extended basis:
// b[r] = t e[r] - a[r] s[r] + gadget[r] s'[r].
void keygen_combine(const DevTables &T, double *b, uint64_t a_stream, const double *e, const double *s_,
                    const double *sp, const double *gadget, hipStream_t s);
// Encryption: noisy = t e + mu (small integers, N values), then
// c0[r] = noisy_eval[r] - a[r] s[r] over the L ciphertext primes.
void enc_noisy(const DevTables &T, double *out, const double *e, const double *mu, hipStream_t s);
void enc_combine(const DevTables &T, double *c0, const double *noisy_eval, const double *a, const double *s_,
                 hipStream_t s);
// Decryption: v[r] = c0 + c1 s (+ c2 s^2) over the L ciphertext primes.
void dec_combine(const DevTables &T, double *v, const double *ct, int comps, const double *s_,
                 const double *s2, hipStream_t s);
// Integer polynomial values (|x| < t/2) times t: out = t * x (used for errors).
void scale_small(double *out, const double *x, double c, int N, hipStream_t s);

}  // namespace hg
