/*
 * hegmm.h -- C ABI of the MI355X (gfx950) HE matrix-multiplication library.
 *
 * Problem (the paper's Section III-A): C_{m x n} = A_{m x l} x B_{l x n} for
 * arbitrary positive m, l, n, computed on encrypted operands.  Clients encrypt
 * A and B, the cloud multiplies the ciphertexts, clients decrypt (Section II-A
 * and the client/cloud split of Algorithm 2: preprocessing on the client,
 * multiplication on the cloud, encrypted result returned).  The cloud-side
 * method is HEGMM-Enhanced (Algorithm 2, Section III-C), built from the SIMD
 * primitives HE-Add, HE-Mult, HE-CMult and HE-Rot over the ring
 * Z_q[X]/(X^N + 1) (Section IV-A), realised here as BGV with hybrid key
 * switching.
 *
 * Conventions common to every call:
 *  - Every function returns hg_status; 0 is success, a negative value an
 *    error, and hg_last_error() then gives a thread-local message.
 *  - Handles (hg_ctx, hg_ct) are opaque and owned by the caller, who frees
 *    them with hg_ctx_destroy / hg_ct_free.  The library never frees caller
 *    memory and keeps no caller pointer after a call returns.
 *  - Host pointers (matrices, serialisation buffers, shapes) are plain host
 *    memory read or written before the call returns.  Ciphertext payloads
 *    live in device memory owned by their hg_ct.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    hg_hegmm / hg_rotate / hg_mul only enqueue work; their outputs are valid
 *    once the stream reaches that point.  Inputs must stay alive until then.
 *  - Matrix entries are signed 64-bit integers reduced mod t (negative values
 *    map to value + t); results are returned in [0, t).
 *  - Not thread safe: one thread per context at a time.
 */
#ifndef HEGMM_H
#define HEGMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hg_status;
enum {
    HG_OK = 0,
    HG_EINVAL = -1,   /* bad argument: non-positive dimension, null pointer, mismatched handles */
    HG_ENOFIT = -2,   /* shape cannot be planned into one ciphertext row, even with inner blocking */
    HG_ENOKEY = -3,   /* a rotation key this shape needs was not generated */
    HG_ENOMEM = -4,   /* device or host allocation failed */
    HG_EDEVICE = -5,  /* HIP runtime error, or no gfx950 device */
    HG_ESTATE = -6    /* call not allowed in this state (e.g. encrypt after hg_drop_secret) */
};

typedef struct hg_ctx hg_ctx;  /* parameters, device tables, device-resident evaluation keys */
typedef struct hg_ct hg_ct;    /* one packed operand/result: nb >= 1 ciphertexts on the device */

/* BGV parameter set over the ring Z_q[X]/(X^N + 1) of Section IV-A.
 * N: ring degree, a power of two in [64, 32768] (rows longer than 16384 use
 * two-pass transforms).  t: plaintext modulus, prime, t = 1 (mod 2N) so that
 * all N/2 slots of a rotation row are usable.  L: ciphertext primes
 * (1..12).  alpha: special primes, also the number of primes per
 * key-switching digit (1..4, L+alpha <= 16).  The primes are the first
 * L+alpha primes below 2^prime_bits that are 1 (mod 2N), in descending
 * order; the alpha largest are the special ones.  The error distribution is
 * the discrete Gaussian of width sigma on [-19, 19].  The paper fixes none of
 * q, t, sigma or the key-switching method (its experiments used a library's
 * defaults); zero-initialised trailing fields select the defaults. */
typedef struct {
    uint32_t N;
    uint64_t t;
    uint32_t L;
    uint32_t alpha;
    uint32_t method;   /* 0 or 2: HEGMM-En (Algorithm 2); 1: HEGMM (Algorithm 1, column- or
                          row-major, no duplication or blocking; for comparison), sigma and
                          tau applied by the client while packing; 3: Algorithm 1 with the
                          operands packed as they are and sigma / tau evaluated on the
                          ciphertexts by the diagonal method (2 min(m,l) - 1 and
                          2 min(n,l) - 1 rotations, Theorems 1 and 2).  HG_EINVAL above 3. */
    uint32_t min_blocks; /* 0 or 1: every product splits its inner dimension into as few
                            blocks as fit one ciphertext (usually one); k > 1: into at
                            least k blocks (at most l), each accumulated into the same
                            result (the blockwise product of Section IV-D, forced; the
                            result decrypts to the same A B, its bits differ).  HEGMM-En
                            only (HG_EINVAL with method 1 or 3). */
    uint32_t relin;    /* 0: lazy relinearisation, once per product on the three-component
                          sum of the loop's tensor products (the default); 1: eager, each
                          tensor product of the loop relinearised on its own (HE-Mult of
                          Section II-A) and the two-component results summed: one key
                          switch per loop product instead of one per product, the same
                          decrypted result, different bits.  Either method.  HG_EINVAL
                          for other values. */
    uint32_t ks_order; /* how a linear transform sum_z u_z (.) Rot(ct, z) (Eq. (lintrans),
                          Section III-B-1: the eps/omega transforms, sigma / tau of method 3,
                          the fold) is composed.  0: the masked key-switching sums of all its
                          rotations are divided by the special modulus P once (the default,
                          fewer transforms); 1: the paper's primitive order, each rotation a
                          complete HE-Rot with its own division by P, then HE-CMult by its
                          mask, then HE-Add.  Same decrypted result, different bits.
                          HG_EINVAL for other values. */
    uint32_t prime_bits; /* 0 (= 50) or 32..50: bit bound of the ciphertext and special
                            primes.  The FP64 residue arithmetic needs primes below 2^50.
                            HG_EINVAL outside that range. */
    double sigma;      /* 0 (= 3.2) or 3.2: width of the discrete Gaussian error; the
                          sampler's cumulative table is fixed for 3.2, other widths are
                          HG_EINVAL. */
} hg_params;

/* Create a context on HIP device `hip_device` (must be gfx950).
 * Errors: HG_EINVAL (parameters out of range), HG_EDEVICE, HG_ENOMEM. */
hg_status hg_ctx_create(const hg_params *params, int hip_device, hg_ctx **out);
void hg_ctx_destroy(hg_ctx *ctx);

/* Device memory of ciphertext handles.  By default every handle the library
 * creates (hg_encrypt, hg_hegmm, hg_hegmm_batch and graph results,
 * hg_ct_import, the primitives) takes its own hipMalloc, and hg_ct_free
 * returns it with hipFree, which waits for the whole device.  A caller can
 * supply the memory instead, for instance from a framework's caching
 * allocator: alloc(bytes, stream, user) returns device memory of at least
 * `bytes` for use on `stream` (the stream of the call that creates the
 * handle; NULL for hg_encrypt, hg_ct_import and graph results), or NULL on
 * failure (the call then fails with HG_ENOMEM); release(ptr, user) takes it
 * back when the handle is freed.  release may be called while work that
 * reads or writes the memory is still queued on that stream, so the
 * allocator must not reuse the memory for work on another stream before that
 * work has finished (stream-ordered caching allocators guarantee this).
 * A handle always goes back to the release function in force when it was
 * created.  Both NULL: back to hipMalloc / hipFree.  Internal workspaces,
 * keys and tables always use the library's own allocations.
 * Errors: HG_EINVAL (only one of alloc, release given). */
typedef void *(*hg_alloc_fn)(size_t bytes, void *stream, void *user);
typedef void (*hg_release_fn)(void *ptr, void *user);
hg_status hg_set_allocator(hg_ctx *ctx, hg_alloc_fn alloc, hg_release_fn release, void *user);

/* Key generation (client role; Section II-A: clients encrypt the source
 * matrices and decrypt the results, and SIMD packing needs the key material
 * for slot rotations).  Samples the secret key from `seed` and
 * generates, on the device, the relinearisation key and every rotation key
 * that the HEGMM-En plans of the given shapes need.  `shapes` holds nshapes
 * triples (m, l, n), row after row.  May be called again to add the keys of
 * more shapes under the same seed.  Errors: HG_EINVAL, HG_ENOFIT (a shape
 * cannot be planned), HG_ESTATE (after hg_drop_secret with a new seed). */
hg_status hg_keygen(hg_ctx *ctx, uint64_t seed, const int32_t *shapes, size_t nshapes);

/* Output blocking (Section IV-D, the blocked product of large matrices):
 * register the partition of shape (m, l, n) -- A's row blocks of rows[0..nrows)
 * rows, B's column blocks of cols[0..ncols) columns, sizes summing to m and n
 * -- before the shape's keys and operands are made.  Without a registered
 * partition a shape whose result does not fit one ciphertext gets the
 * fewest blocks (at most 4096) of near-equal sizes whose block products each
 * fit, else HG_ENOFIT.  Every block product must fit one ciphertext (its
 * inner dimension is split as it needs, with one accumulator).  HEGMM-En
 * only.  hg_encrypt, hg_hegmm, hg_hegmm_batch and hg_decrypt take
 * output-blocked shapes; recorded batches (hg_graph_create), the request
 * server and hg_hegmm_noalloc do not.
 * Errors: HG_EINVAL (sizes, a shape planned already as one product, more
 * than 4096 blocks), HG_ENOFIT (a block product does not fit). */
hg_status hg_set_partition(hg_ctx *ctx, int m, int l, int n, const int32_t *rows, int nrows, const int32_t *cols,
                           int ncols);

/* The partition of shape (m, l, n): out = {nrows, ncols, rows..., cols...};
 * a shape that fits one ciphertext reports {1, 1, m, n}.  *count receives the
 * number of values; out may be NULL to query it.
 * Errors: HG_EINVAL (buffer too small), HG_ENOFIT. */
hg_status hg_get_partition(hg_ctx *ctx, int m, int l, int n, int32_t *out, size_t cap, size_t *count);

/* Forget the secret key (server role; the cloud of Section II-A computes on
 * ciphertexts only): evaluation keys stay, encrypt and
 * decrypt then fail with HG_ESTATE while hg_hegmm still works. */
hg_status hg_drop_secret(hg_ctx *ctx);

/* Client preprocessing of Algorithm 2: pack one operand of the product
 * A (m x l) x B (l x n) for the cloud and encrypt it.  role 0: X points to
 * A (row-major m x l); role 1: X points to B (row-major l x n).  The packing
 * depends on the whole shape (duplication count, orientation, inner
 * blocking).  A product whose m x n result does not fit one ciphertext is an
 * output-blocked product (the blocked matrix multiplication of Section
 * IV-D): A is split into row blocks and B into column blocks (the shape's
 * partition, see hg_set_partition), block k = (i, j), row-major over the
 * partition, is the ordinary product A_i (rows_i x l) x B_j (l x cols_j), and
 * the handle holds, for every k in turn, the packed operand of that product
 * encrypted with nonce nonce * 65536 + k (nonce < 2^47).  `nonce` selects the
 * encryption randomness; the same (role, nonce, shape) must not be reused for
 * different data.  *out receives a new handle.  Errors: HG_EINVAL,
 * HG_ENOFIT, HG_ESTATE. */
hg_status hg_encrypt(hg_ctx *ctx, int role, const int64_t *X, int m, int l, int n,
                     uint64_t nonce, hg_ct **out);

/* Cloud multiplication of Algorithm 2 (HEGMM-En) on encrypted operands made
 * by hg_encrypt for the same (m, l, n).  *ctC receives a new result handle;
 * the work is enqueued on `stream`.  An output-blocked product runs all its
 * block products in one batch and its result holds one ciphertext per
 * block, in block order.  Errors: HG_EINVAL (shape differs from the
 * operands'), HG_ENOFIT, HG_ENOKEY, HG_EDEVICE. */
hg_status hg_hegmm(hg_ctx *ctx, const hg_ct *ctA, const hg_ct *ctB, int m, int l, int n,
                   hg_ct **ctC, void *stream);

/* hg_hegmm for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * product is the one hg_hegmm computes for the same operands, bit for bit,
 * written into the caller's existing handle ctC, which must hold one
 * two-component ciphertext at the full level (an earlier hg_hegmm result of
 * any shape, or hg_ct_import(..., 1, 2, ...) of any valid words) and must not
 * be one of the operands; its words are overwritten and it becomes the
 * result of shape (m, l, n).  The call allocates nothing: every workspace
 * (accumulators, hoisted digits, inner-product sums, the division by P,
 * descriptor tables) lies in one fixed device array of
 * HG_NOALLOC_SCRATCH_BYTES (96 MiB) that each GPU the library runs on holds
 * from the library's first use there until the process ends, and the tables
 * are staged through 1 MiB of pinned host memory that hg_ctx_create made for
 * the context.  Nothing in the workspace needs to start at zero.  All calls
 * on one GPU share that array (it keeps the last call's contents): calls
 * that overlap on one GPU race -- from two streams, two threads or two
 * contexts -- so order them on one stream.  Enqueued on `stream` like
 * hg_hegmm; timing (hg_set_timing) and the "pipeline" knob do not apply.
 * Errors: HG_EINVAL (as hg_hegmm, a result handle of the wrong form, or a
 * product whose workspace exceeds the array or whose tables exceed the
 * staging; nothing is enqueued then), HG_ESTATE (the shape was not listed in
 * hg_keygen, so its plan and masks do not exist yet), HG_ENOKEY. */
#define HG_NOALLOC_SCRATCH_BYTES (96ull << 20)
hg_status hg_hegmm_noalloc(hg_ctx *ctx, const hg_ct *ctA, const hg_ct *ctB, int m, int l, int n, hg_ct *ctC,
                           void *stream);

/* Many independent HE matmuls of (possibly) different shapes in one call
 * (Algorithm 2 per request; the random shape pairs of Section IV-B as one
 * batch).
 * mln holds cnt triples.  The products share the launches of each phase
 * (one hoisting launch, one key-switching launch, ...), and rotations that
 * several products need read each key once per launch.  C[i] receives new
 * handles.  Errors as hg_hegmm; every request is checked before any work
 * is enqueued, so on an error no handle is returned and nothing of this
 * call runs on the stream. */
hg_status hg_hegmm_batch(hg_ctx *ctx, size_t cnt, const hg_ct *const *A, const hg_ct *const *B,
                         const int32_t *mln, hg_ct **C, void *stream);

/* Record a batch (the launches hg_hegmm_batch would make for it) once as a
 * HIP graph with private workspaces, for replay with no host work.  The
 * graph binds the operand handles and the new result handles C[i]: every
 * hg_graph_launch recomputes C[i] from the current contents of A[i], B[i]
 * (refresh them with hg_ct_load).  Bound handles must stay alive until
 * hg_graph_destroy.  Recording runs the batch once eagerly first (C[i] then
 * already hold the products).  Errors as hg_hegmm_batch. */
typedef struct hg_graph hg_graph;
hg_status hg_graph_create(hg_ctx *ctx, size_t cnt, const hg_ct *const *A, const hg_ct *const *B,
                          const int32_t *mln, hg_ct **C, hg_graph **out);
/* Enqueue one replay on `stream`.  Replays of one graph must not overlap:
 * launch them on one stream, or order them. */
hg_status hg_graph_launch(hg_graph *g, void *stream);
void hg_graph_destroy(hg_graph *g);

/* Overwrite a handle's contents with canonical words (the hg_ct_export
 * layout of a handle of the same size), keeping its shape and role; used to
 * feed new operands to a recorded graph.  Synchronises `stream`.  Errors:
 * HG_EINVAL (word count, residue range). */
hg_status hg_ct_load(hg_ctx *ctx, hg_ct *ct, const uint64_t *buf, size_t nwords, void *stream);

/* Decrypt (client role: the encrypted result returned by the cloud, the last
 * step of Algorithm 2; Section II-A) a result made by hg_hegmm for shape
 * (m, l, n) -- or the
 * hg_ct_import (two components, one ciphertext, or one per output block of
 * an output-blocked shape) of its exported words, such as a served result --
 * and unpack it into C (row-major m x n, values in [0, t)); output blocks are
 * placed at their rows and columns.  Synchronises the device.  Errors:
 * HG_EINVAL (a packed operand or a result of another shape), HG_ESTATE. */
hg_status hg_decrypt(hg_ctx *ctx, const hg_ct *ctC, int m, int l, int n, uint64_t *C);

/* Canonical serialisation: coefficient form, residues in [0, q_i), the
 * ciphertexts of the handle in order, each component c0 then c1 (then c2),
 * each limb q_0..q_{L-1} (q_0..q_{l-1} for a handle switched to level l by
 * hg_mod_switch), N little-endian u64 words per limb.  *needed gets
 * the word count; buf may be NULL to query it.  Errors: HG_EINVAL (buffer
 * too small). */
hg_status hg_ct_export(hg_ctx *ctx, const hg_ct *ct, uint64_t *buf, size_t nwords, size_t *needed);

/* Rebuild a handle from hg_ct_export output (ncts ciphertexts of
 * `components` components each, all L limbs).  Words must be residues in
 * [0, q_i).
 * Errors: HG_EINVAL. */
hg_status hg_ct_import(hg_ctx *ctx, const uint64_t *buf, size_t nwords, int ncts, int components,
                       hg_ct **out);

void hg_ct_free(hg_ct *ct);

/* ---- single-ciphertext primitives (Section II-A set) ----------------- */

/* Encrypt / decrypt a raw slot vector (row 0: S = N/2 values mod t; row 1 is
 * zero).  Errors: HG_EINVAL, HG_ESTATE. */
hg_status hg_encrypt_slots(hg_ctx *ctx, const int64_t *slots, uint64_t nonce, hg_ct **out);
hg_status hg_decrypt_slots(hg_ctx *ctx, const hg_ct *ct, uint64_t *slots);

/* HE-Rot: left rotation of the slots by z (negative z rotates right).  Needs
 * the rotation key of z (generated by hg_keygen_rotations or as part of a
 * shape's plan).  Errors: HG_ENOKEY, HG_EINVAL. */
hg_status hg_rotate(hg_ctx *ctx, const hg_ct *ct, int z, hg_ct **out, void *stream);

/* Generate rotation keys for explicit amounts (client role). */
hg_status hg_keygen_rotations(hg_ctx *ctx, const int32_t *z, size_t count);

/* HE-Mult: tensor product followed by relinearisation. */
hg_status hg_mul(hg_ctx *ctx, const hg_ct *a, const hg_ct *b, hg_ct **out, void *stream);

/* HE-Add. */
hg_status hg_add(hg_ctx *ctx, const hg_ct *a, const hg_ct *b, hg_ct **out, void *stream);

/* HE-CMult by a 0/1 (or any mod-t) slot vector of length S. */
hg_status hg_cmul(hg_ctx *ctx, const hg_ct *a, const int64_t *slots, hg_ct **out, void *stream);

/* BGV modulus switching of a two-component handle (an hg_hegmm result, any
 * number of ciphertexts): a new handle at `drop` primes fewer, q_0..q_{l-1}
 * with l = L - drop (1 <= drop < L), that decrypts to the same plaintext, so
 * a result goes back to the client in l/L of the words.  Each step from
 * level l to l - 1 scales the ciphertext by q_{l-1} mod t and divides it by
 * q_{l-1} with the t-corrected rounding of the division by P (the standard
 * BGV rescaling; the scaling keeps the plaintext unscaled).  The new handle
 * can be exported (hg_ct_export writes l limbs per component), loaded
 * (hg_ct_load) and decrypted (hg_decrypt), but is no operand of any other
 * call (HG_EINVAL).  Enqueued on `stream`, which it synchronises before it
 * returns.  Errors: HG_EINVAL (not two components, drop out of range, an
 * input already switched to fewer than drop + 1 primes), HG_ENOMEM. */
hg_status hg_mod_switch(hg_ctx *ctx, const hg_ct *ct, int drop, hg_ct **out, void *stream);

/* ---- serving: continuous batching ------------------------------------ */

/* A request loop on its own thread, for the cloud side of Algorithm 2 under
 * a stream of independent products of mixed shapes.  Clients submit the
 * serialised operands (hg_ct_export words of hg_encrypt outputs for that
 * shape; what a client sends to the cloud).  The server admits queued
 * requests in arrival order while its modelled device memory stays within
 * hbm_budget: the workspace every lane keeps (sized for the largest group it
 * ran) plus the buffers of the groups in flight, each request modelled by
 * hg_request_footprint (its buffers are released when its group finishes,
 * its workspace share stays with the lane).  It launches each
 * admitted group through the batched executor on one of `lanes` streams so
 * that groups overlap on the device, and admits new arrivals as soon as a
 * lane and budget are free.  Keys stay resident in the context.  Each result
 * is bit-identical to hg_hegmm of the same operands alone.
 * While a server exists its thread owns the context: the caller may use only
 * hg_server_* and hg_request_footprint on it until hg_server_destroy, which
 * finishes every submitted request first; every other call on the context
 * (or on a graph recorded from it), and a second hg_server_create, returns
 * HG_ESTATE.  hg_ct_free stays allowed.  hg_server_submit and hg_server_wait
 * may be called from several threads. */
typedef struct hg_server hg_server;
typedef struct {
    int32_t max_batch;     /* products per launch group, >= 1 */
    int32_t lanes;         /* launch groups in flight at once, 1..8, one stream each */
    uint64_t hbm_budget;   /* bytes of modelled footprint admitted at once; 0 = no limit.
                              A request larger than the budget still runs when nothing else does. */
} hg_server_config;

/* Errors: HG_EINVAL (configuration out of range), HG_ESTATE (a server owns
 * the context already), HG_EDEVICE. */
hg_status hg_server_create(hg_ctx *ctx, const hg_server_config *cfg, hg_server **out);

/* Queue one product.  a_words / b_words: nb * 2 * L * N words each (nb the
 * shape's inner block count), residues in [0, q_i); copied before return.
 * *ticket identifies the request.  Errors: HG_EINVAL (word count, residue
 * range, dimensions), HG_ENOKEY (shape not listed in hg_keygen). */
hg_status hg_server_submit(hg_server *srv, const uint64_t *a_words, size_t a_nwords, const uint64_t *b_words,
                           size_t b_nwords, int m, int l, int n, uint64_t *ticket);

/* Block until the request is done.  c_words (may be NULL) receives the
 * result's hg_ct_export words (2 * L * N, one ciphertext of the shape's
 * result; hg_ct_import with ncts 1, components 2 gives a handle for
 * hg_decrypt).  times3 (may be NULL) receives the submit, start and done
 * times in seconds since the server was created; done is when the result was
 * back in host memory.  A ticket can be waited for once.  Errors: HG_EINVAL
 * (unknown ticket, buffer too small), or the error of the request's launch. */
hg_status hg_server_wait(hg_server *srv, uint64_t ticket, uint64_t *c_words, size_t c_nwords, double *times3);

/* Hold (paused = 1) or resume (paused = 0) admission.  While held, submitted
 * requests queue up and groups already launched finish; on resume the queue
 * is admitted in arrival order as usual (a burst fills whole groups and
 * several lanes at once).  hg_server_destroy resumes by itself.
 * Errors: HG_EINVAL. */
hg_status hg_server_pause(hg_server *srv, int paused);

/* out8: completed requests, launch groups, mean group size, peak modelled
 * device bytes (kept workspaces plus buffers in flight), peak groups in
 * flight, queued requests, modelled device bytes now, seconds since
 * creation. */
hg_status hg_server_stats(hg_server *srv, double *out8);

/* Finish every submitted request, stop the thread, release the lanes. */
void hg_server_destroy(hg_server *srv);

/* Modelled device bytes that one product of this shape holds while it runs
 * on a server lane: its operands as received and in evaluation form, its
 * result, its accumulator and its share of the pass workspace (hoisted
 * digits, inner-product sums, division-by-P buffers), plus 3 MiB for the
 * rounding of workspaces and the descriptor tables.  An upper bound of the
 * device memory the product adds to its group.
 * Errors: HG_EINVAL, HG_ENOFIT. */
hg_status hg_request_footprint(hg_ctx *ctx, int m, int l, int n, uint64_t *bytes);

/* ---- tuning ----------------------------------------------------------- */

/* Set an execution knob of the context (used by the autotuner; results are
 * bit-identical for every setting).  Knobs belong to the context: other
 * contexts keep theirs.  Not while a server owns the context (HG_ESTATE).
 * Names:
 *   "pipeline"   chunks (1..16) of a pass whose inner products overlap the
 *                division by P of the previous chunk on a second stream
 *                (1: no overlap, one stream)
 *   "fuse_rows"  passes with at most this many rows per transform chain run
 *                the fused one-workgroup-per-row kernels (alpha = 1 only)
 *   "ip_chunk"   key-switched terms that share a key per workgroup of the
 *                key-stationary inner products (one launch per round of
 *                terms), used for passes whose keys repeat at least four
 *                times on average; 0 (the default) disables key grouping
 *   "ip_order"   1: the plain (one launch) inner products start their jobs
 *                ordered by their keys, so jobs that read the same keys run
 *                together; 0: in pass order
 *   "split_rows" transforms of fewer rows than this split each row over
 *                N/1024 workgroups (two passes)
 *   "half_rows"  fused transform chains (few-row passes) of at most this many
 *                rows run two workgroups per row, each finishing one half of
 *                the forward transform (default 128; 0: off)
 *   "ntt_radix"  radix of the one-workgroup row transforms of 4096- and
 *                8192-point rows: 8, 16, or 0 for the built-in choice (8)
 *   "xcd_rows"   1 (default): one-workgroup forward transforms hand each
 *                XCD a contiguous block of rows, so rows reading the same
 *                input row share an L2; 0: rows in workgroup order
 *   "batch_window" products per launch group inside hg_hegmm_batch
 *                (0: all at once; default 64, 16 for N >= 16384)
 * Errors: HG_EINVAL (unknown name, negative value, "pipeline" outside
 * [1, 16], "ntt_radix" other than 0, 8, 16, "xcd_rows" other than 0, 1). */
hg_status hg_tune(hg_ctx *ctx, const char *name, int64_t value);

/* ---- introspection ---------------------------------------------------- */

/* Plan of a shape: out[0..9] = transposed, nb, lb, d, M, K, W, rotations,
 * masked diagonals, key-switched terms. Errors: HG_EINVAL, HG_ENOFIT. */
hg_status hg_plan_info(hg_ctx *ctx, int m, int l, int n, int64_t *out10);

/* The primes of the context: out[0..L-1] = q_0.., out[L..L+alpha-1] = p_0.. */
hg_status hg_primes(hg_ctx *ctx, uint64_t *out);

/* Per-phase timing of the last hg_hegmm / hg_hegmm_batch call (of its last
 * launch window) in milliseconds, measured with HIP events on its stream
 * (out[0..8]: hoist, inner products, division by P, tensor/accumulate,
 * relinearise, fold, total, the mean duration of one inner-product launch of
 * the transform pass, and the number of those launches).  With pipelining
 * the inner-product and division phases overlap: out[1] ends with the last
 * inner-product launch and out[2] with the last division.  Only filled when
 * timing was enabled with hg_set_timing(ctx, 1); synchronises the stream.
 * hg_set_timing(ctx, 2) instead times only the transform-pass inner-product
 * launches, with start / stop events carried by the dispatches themselves
 * (no markers between kernels and no synchronisation per call), and the
 * forward-transform launches of that pass's division by P (when it runs
 * unfused), kept across calls until hg_launch_timing reads them: out[0] =
 * mean inner-product launch duration in ms, out[1] = number of those
 * launches, out[2] / out[3] the same for the forward transforms; it waits for
 * them and starts a new tally.  At most 65536 calls' launches are kept until
 * read; later ones are not timed.
 * 0 turns timing off; launches recorded into a graph are never timed.
 * Errors: HG_EINVAL (mode outside 0..2). */
hg_status hg_set_timing(hg_ctx *ctx, int enable);
hg_status hg_last_timing(hg_ctx *ctx, double *out9);
hg_status hg_launch_timing(hg_ctx *ctx, double *out4);

/* ---- measurement ------------------------------------------------------ */

/* Rate of modular products on device `device` (the measurement behind the
 * library's FP64 residue arithmetic): blocks x 256 threads, each running 4
 * independent chains x <- x w mod q of `iters` products, `reps` launches
 * timed with HIP events after one warm-up.  form 0: the FP64 product every
 * kernel uses; 1: 64-bit integer Shoup product (precomputed w'); 2: 64-bit
 * integer Barrett product.  q: an odd modulus in (2^49, 2^50).  *out_per_s:
 * products per second; *checksum (may be NULL): an xor of results.
 * Allocates and frees its own buffer; synchronises the device.
 * Errors: HG_EINVAL, HG_EDEVICE, HG_ENOMEM. */
hg_status hg_bench_modmul(int device, int form, uint64_t q, int blocks, int iters, int reps, double *out_per_s,
                          uint64_t *checksum);

/* Plain HBM streaming on `device` over a buffer of `bytes` (>= 1 MiB):
 * mode 0 reads it (16-byte loads, 8 workgroups per CU, grid-stride), mode 1
 * copies it into a second buffer; `reps` launches after one warm-up.
 * *out_bytes_per_s counts bytes read plus bytes written.  The practical
 * ceiling the memory-bound inner products are compared with.
 * Errors: HG_EINVAL, HG_EDEVICE, HG_ENOMEM. */
hg_status hg_bench_stream(int device, size_t bytes, int mode, int reps, double *out_bytes_per_s);

const char *hg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
