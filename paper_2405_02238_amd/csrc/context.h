// Library context: parameters, device tables, keys, plans, workspaces.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <atomic>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "kernels.h"
#include "planner.h"

namespace hg {

// Error carrying an hg_status code.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void hip_check(hipError_t e, const char *what);
#define HGCHK(x) ::hg::hip_check((x), #x)

struct Ctx;

// Caller-supplied device memory for ciphertext handles (hg_set_allocator):
// alloc(bytes, stream, user) -> device memory or null; release(ptr, user).
typedef void *(*CtAllocFn)(size_t bytes, void *stream, void *user);
typedef void (*CtReleaseFn)(void *ptr, void *user);

// A packed operand/result: ncts ciphertexts of `comps` components, each
// comps x L x N doubles in evaluation form, one device allocation.
struct Ct {
    Ctx *ctx = nullptr;
    int ncts = 1, comps = 2;
    int m = 0, l = 0, n = 0;   // shape (0 for raw slot ciphertexts)
    int side = -1;             // packed side (0 left, 1 right, 2 result, -1 raw)
    int level = 0;             // ciphertext primes per component (0: all L; fewer after modulus switching)
    double *d = nullptr;
    bool owns = true;          // false: a view into memory owned elsewhere
    CtReleaseFn release = nullptr;   // d came from the caller's allocator: give it back here
    void *release_user = nullptr;
    int lv() const;            // ciphertext primes per component
    size_t words() const;      // doubles in total
    double *ct(int i) const;   // start of ciphertext i
    ~Ct();
};

struct PlanEntry {
    Plan plan;
    std::vector<const double *> mask_ptrs;   // device masks, plan.masks order
    // every rotation key the plan needs was found once (keys are only ever
    // added to a context, so the check need not be repeated; set from the
    // serving thread and the submitting thread alike)
    mutable std::atomic<bool> keys_found{false};
};

// Per-stream scratch arena, grown on demand.
struct Arena {
    void *base = nullptr;
    size_t cap = 0;
    size_t used = 0;
    void *pinned = nullptr;      // host staging for descriptor tables: `ring` slots of pinned_cap bytes
    void *pinned_dev = nullptr;  // the same memory as the device addresses it
    size_t pinned_cap = 0;
    hipEvent_t staged = nullptr; // completion of the copy out of the ring's last slot (ring 1: of every copy)
    // Stream arenas stage call after call in a ring of slots, one stream
    // ordering every copy, so only the copy out of the last slot carries a
    // completion signal (a dispatch the host can wait on ends with a
    // system-scope release, a few microseconds), and the host waits on it
    // before it writes the first slot again.  Graph and fixed arenas keep
    // one slot: a graph replays the bytes of its slot, a fixed arena is used
    // from any stream.
    int ring = 1;
    int slot = 0;                // the slot the next call writes
    uint64_t copies = 0;         // copies out of the ring since it was made
    void *acc = nullptr;         // per-call accumulators (3 x L x N per product, R for folds)
    size_t acc_cap = 0;
    // A fixed arena (fixed_bytes > 0) never grows: each call places its
    // accumulators at fixed_base and its pass scratch right after them, and
    // a call that needs more than fixed_bytes (or more descriptor-table
    // staging than pinned_cap) fails before it enqueues anything.  Its device
    // memory belongs to someone else and is not freed here.
    char *fixed_base = nullptr;
    size_t fixed_bytes = 0;
    bool exact = false;          // grow to the size needed (rounded to 1 MiB), without headroom
    void release();              // free everything (device must be idle)
};

struct Timing {
    bool enabled = false;
    double ms[9] = {0};
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ip_pairs;   // transform-pass inner-product launches
    std::vector<std::pair<hipEvent_t, hipEvent_t>> md_pairs;   // its division's forward-transform launches
    bool pooled = false;   // ip_pairs take events from Ctx::lt_event (kept until read) instead of the ring
};

// Per user stream: the second stream of the pipelined passes and two rings
// of reusable events (ordering, timing).
struct StreamAux {
    hipStream_t side = nullptr;
    std::vector<hipEvent_t> ev[2];
    size_t next[2] = {0, 0};
};

struct Ctx {
    int device = 0;
    int N = 0, logN = 0, L = 0, alpha = 0, beta = 0, nExt = 0, S = 0;
    uint64_t t = 0, zeta = 0;
    std::vector<uint64_t> qs;     // extended basis: q_0..q_{L-1}, p_0..p_{alpha-1}
    DevTables T;                  // device tables (pointers)
    // Modulus switching from level l to l - 1 (index l = 2..L): the tables of
    // the division by P with P = q_{l-1} (one special prime) over q_0..q_{l-2}.
    std::vector<DevTables> ms_tabs;
    std::vector<void *> owned;    // device allocations released at destroy

    // keys
    bool has_secret = false;
    uint64_t seed = 0;
    double *s_eval = nullptr;     // nExt x N, evaluation form
    double *s2_eval = nullptr;    // L x N (s^2 over Q)
    // A switching key keeps only b_j (beta planes of nExt x N, evaluation
    // form); a_j is regenerated from its stream wherever it is needed.
    double *relin_key = nullptr;
    std::map<const double *, std::vector<uint64_t>> key_streams;   // key -> beta stream states
    std::map<int, double *> rot_keys;   // Galois element -> key
    std::vector<double *> key_of_g;     // the same indexed by Galois element (2N entries, null: none)
    double *rot_key(int g) const { return g > 0 && g < (int)key_of_g.size() ? key_of_g[g] : nullptr; }
    size_t key_words() const { return (size_t)beta * nExt * N; }

    // plans and masks
    std::map<std::tuple<int, int, int>, std::unique_ptr<PlanEntry>> plans;
    // Output blocking (Section IV-D) of products whose result does not fit
    // one ciphertext: row sizes of A's blocks, then column sizes of B's.
    struct Partition {
        std::vector<int> rows, cols;
        int blocks() const { return (int)(rows.size() * cols.size()); }
    };
    std::map<std::tuple<int, int, int>, Partition> partitions;   // registered or chosen, per shape
    // The partition of a shape if its result needs output blocks (nullptr
    // when one ciphertext holds it); chosen on first use unless registered.
    const Partition *partition_for(int m, int l, int n);
    // Register a partition (every block must be plannable; sizes sum to m, n).
    void set_partition(int m, int l, int n, const std::vector<int> &rows, const std::vector<int> &cols);
    bool plannable(int m, int l, int n) const;
    std::map<std::string, double *> mask_cache;   // slot bitmap -> device mask (nExt x N)

    std::map<hipStream_t, Arena> arenas;
    // Graph recording: while `capture_arenas` is set, every launch window
    // takes the next arena of that list (private to the graph, kept for its
    // replays) instead of the stream's; while `capturing`, nothing may
    // synchronise or allocate.
    std::vector<std::unique_ptr<Arena>> *capture_arenas = nullptr;
    size_t capture_next = 0;
    bool capturing = false;
    // While set, every launch window uses this arena (the fixed workspace of
    // the allocation-free entry point) instead of the stream's.
    Arena *fixed_arena = nullptr;
    Arena noalloc_arena;          // staging and device views of that workspace
    Arena &arena_for(hipStream_t st);
    Timing timing;
    // Launch timing (hg_set_timing mode 2): the transform-pass inner-product
    // launches of every call record start / stop events carried by the
    // dispatch itself, kept across calls without synchronising; read and
    // recycled by hg_launch_timing.
    // At most LT_MAX launches are kept until read; later ones go untimed.
    static constexpr size_t LT_MAX = 1 << 16;
    bool launch_timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> lt_pairs;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> lt_md_pairs;   // forward transforms of the division by P
    std::vector<hipEvent_t> lt_free;
    hipEvent_t lt_event();
    int min_blocks = 1;   // inner blocks of every plan at least this many (fixed at creation)
    // the caller's allocator for ciphertext handles (null: hipMalloc / hipFree)
    CtAllocFn ct_alloc_fn = nullptr;
    CtReleaseFn ct_release_fn = nullptr;
    void *ct_alloc_user = nullptr;
    // device memory for the words of handle c, to be used on stream st
    void ct_alloc(Ct *c, hipStream_t st);
    int fuse_rows = 256;  // passes with at most this many rows per chain use the fused kernels
    int ip_chunk = 0;     // terms sharing a key per workgroup in the key-stationary inner products (0: off)
    int ip_order = 1;     // plain inner products launch their jobs ordered by key (0: pass order)
    int batch_window = 64; // products per launch group in hegmm_batch (0: all)
    int pipeline = 1;      // chunks of a pass whose inner products and division by P overlap (1: off)
    std::map<hipStream_t, StreamAux> aux;
    hipStream_t side_stream(hipStream_t st);
    hipEvent_t event(hipStream_t st, bool timing);

    int method = 2;        // 2: HEGMM-En; 1: the paper's Algorithm 1
    int relin = 0;         // 0: one relinearisation per product; 1: one per loop product (eager)
    // 0: a linear transform's masked key-switched terms are summed and divided
    // by P once; 1: each rotation is divided by P on its own and masked after
    // (the paper's HE-Rot, HE-CMult, HE-Add order)
    int ks_order = 0;
    int servers = 0;       // request loops (hg_server) that own this context now
    int prime_bits = 50;   // ciphertext and special primes lie below 2^prime_bits
    Ctx(uint32_t N, uint64_t t, uint32_t L, uint32_t alpha, int device, int method = 2, int prime_bits = 50);
    ~Ctx();

    double *dev_alloc(size_t words);
    const PlanEntry &plan_for(int m, int l, int n);

    void keygen(uint64_t seed, const std::vector<int> &galois);
    void drop_secret();
    int galois_of(int z) const;   // 5^(z mod S) mod 2N
    std::vector<int> galois_tab;  // galois_of for z in [0, S)

    // encode slot values (S values in [0, t)) into a centered-lifted plaintext
    // polynomial (N doubles, coefficient form) on `st`
    void encode_slots(const std::vector<uint64_t> &slots, double *mu, hipStream_t st);
    double *mask_for(const std::vector<uint8_t> &bitmap);

    Ct *encrypt_slots(const std::vector<uint64_t> &slots, int side, int block, uint64_t nonce,
                      Ct *into = nullptr, int into_index = 0);
    Ct *encrypt_matrix(int role, const int64_t *X, int m, int l, int n, uint64_t nonce);
    // pack and encrypt one product's operand into ciphertexts [first, first + nb) of `into`
    void encrypt_matrix_into(int role, const int64_t *X, int m, int l, int n, uint64_t nonce, Ct *into, int first);
    // an output-blocked operand: for block k = (i, j) (row-major over the
    // partition) the operand of product (rows[i], l, cols[j]) with nonce
    // nonce * 65536 + k, the blocks' ciphertexts one after another
    Ct *encrypt_blocked(int role, const int64_t *X, int m, int l, int n, uint64_t nonce, const Partition &pt);
    std::vector<uint64_t> decrypt_poly(const Ct &c, int index);   // mu in [0, t), N values
    std::vector<uint64_t> decrypt_slot_values(const Ct &c, int index);

    // cloud side
    struct Request {
        const Ct *A;
        const Ct *B;
        int m, l, n;
        Ct *out;
    };
    const PlanEntry &check_request(const Request &r);   // throws on any invalid request
    void hegmm_batch(std::vector<Request> &reqs, hipStream_t st);
    void hegmm_batch_window(std::vector<Request> &reqs, hipStream_t st);
    Ct *rotate(const Ct &c, int z, hipStream_t st);
    Ct *mul(const Ct &a, const Ct &b, hipStream_t st);
    Ct *add(const Ct &a, const Ct &b, hipStream_t st);
    Ct *cmul(const Ct &a, const std::vector<uint64_t> &slots, hipStream_t st);
    // BGV modulus switching of a two-component ciphertext: drop its last `drop` primes
    Ct *mod_switch(const Ct &c, int drop, hipStream_t st);
    void need_full_level(const Ct &c) const;   // throws unless c has all L primes

    void export_ct(const Ct &c, uint64_t *buf, hipStream_t st);
    Ct *import_ct(const uint64_t *buf, int ncts, int comps, hipStream_t st);
    // overwrite a handle's contents with canonical words (same layout as export)
    void load_ct(Ct &c, const uint64_t *buf, size_t nwords, hipStream_t st);

    // canonical (coefficient form, [0,q)) residues of an L-row polynomial
    // (rows cycle over the first `per` primes; 0: L)
    std::vector<uint64_t> to_host_canonical(const double *eval_rows, int rows, hipStream_t st, int per = 0);

    Arena &arena(hipStream_t st);
};

// A batch of products recorded once as a HIP graph (every launch of its
// windows, with private workspaces and descriptor tables) and replayed with
// no host work: each replay recomputes the bound outputs from the current
// contents of the bound operands.
struct Graph {
    Ctx *C = nullptr;
    hipStream_t gs = nullptr;                    // recording stream
    std::vector<std::unique_ptr<Arena>> arenas;  // one per launch window, kept for the replays
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    Graph(Ctx &c, std::vector<Ctx::Request> &reqs);
    void launch(hipStream_t st);
    ~Graph();
};

}  // namespace hg
