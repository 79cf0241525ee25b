// Library context: parameter set-up, key generation, encryption, decryption
// and the cloud-side HEGMM-En executor.
#include "context.h"

#include <algorithm>
#include <cstring>
#include <numeric>
#include <set>

#include "host_math.h"

namespace hg {

void hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess) {
        if (e == hipErrorOutOfMemory) throw Error(-4, std::string("out of device memory in ") + what);
        throw Error(-5, std::string(hipGetErrorString(e)) + " in " + what);
    }
}

// ---------------------------------------------------------------------------
// random streams (SplitMix64 finaliser; one stream per sampled object)
// ---------------------------------------------------------------------------

namespace {

constexpr uint64_t TAG_SECRET = 1, TAG_RELIN = 2, TAG_ROT = 3, TAG_ENC = 4;

uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// starting state of the stream of object (tag, idx) under a master seed
uint64_t stream_state(uint64_t master, uint64_t tag, uint64_t idx) {
    return mix64(mix64(mix64(master) ^ tag) ^ idx);
}

uint64_t enc_index(int side, int block, uint64_t nonce) {
    return nonce * 4096ULL + (uint64_t)block * 4ULL + (uint64_t)side;
}

double centered_d(uint64_t x, uint64_t m) { return (double)centered_of(x, m); }

}  // namespace

// ---------------------------------------------------------------------------
// Ct
// ---------------------------------------------------------------------------

int Ct::lv() const { return level > 0 ? level : ctx->L; }
size_t Ct::words() const { return (size_t)ncts * comps * lv() * ctx->N; }
double *Ct::ct(int i) const { return d + (size_t)i * comps * lv() * ctx->N; }
Ct::~Ct() {
    if (!d || !owns) return;
    if (release) release(d, release_user);
    else (void)hipFree(d);
}

void Ctx::ct_alloc(Ct *c, hipStream_t st) {
    if (!ct_alloc_fn) {
        c->d = dev_alloc(c->words());
        return;
    }
    void *p = ct_alloc_fn(std::max<size_t>(c->words(), 32) * sizeof(double), (void *)st, ct_alloc_user);
    if (!p) throw Error(-4, "the caller's allocator returned no memory");
    c->d = (double *)p;
    c->release = ct_release_fn;
    c->release_user = ct_alloc_user;
}

// ---------------------------------------------------------------------------
// set-up
// ---------------------------------------------------------------------------

Ctx::Ctx(uint32_t N_, uint64_t t_, uint32_t L_, uint32_t alpha_, int device_, int method_, int prime_bits_) {
    if (method_ < 1 || method_ > 3) throw Error(-1, "method must be 1, 2 or 3");
    method = method_;
    if (N_ < 64 || N_ > 32768 || (N_ & (N_ - 1))) throw Error(-1, "N must be a power of two in [64, 32768]");
    if (L_ < 1 || L_ > 12 || alpha_ < 1 || alpha_ > 4 || L_ + alpha_ > 16)
        throw Error(-1, "need 1 <= L <= 12, 1 <= alpha <= 4, L + alpha <= 16");
    if (t_ < 3 || t_ >= (1ULL << 30) || !is_prime_u64(t_) || (t_ - 1) % (2 * N_) != 0)
        throw Error(-1, "t must be a prime below 2^30 with t = 1 (mod 2N)");
    // FP64 residues need q < 2^50 (arith.h); every prime must exceed t
    if (prime_bits_ < 32 || prime_bits_ > 50) throw Error(-1, "prime_bits must be in [32, 50]");
    prime_bits = prime_bits_;
    device = device_;
    HGCHK(hipSetDevice(device));
    hipDeviceProp_t prop;
    HGCHK(hipGetDeviceProperties(&prop, device));
    if (std::string(prop.gcnArchName).find("gfx950") == std::string::npos)
        throw Error(-5, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
    N = (int)N_;
    logN = 0;
    while ((1 << logN) < N) ++logN;
    L = (int)L_;
    alpha = (int)alpha_;
    beta = (L + alpha - 1) / alpha;
    nExt = L + alpha;
    S = N / 2;
    // 5^z mod 2N for every z in [0, S): looked up for every term of every pass
    galois_tab.resize(S);
    galois_tab[0] = 1;
    for (int z = 1; z < S; ++z) galois_tab[z] = (int)((5ULL * (uint64_t)galois_tab[z - 1]) % (2ULL * (uint64_t)N));
    t = t_;
    // products per launch window of a batch: large rings keep fewer products'
    // hoisted digits in flight (their inner products gather them from cache;
    // measured on 16384-point rings: 16 per window 0.38 against 64 per window
    // 0.41 ms per product)
    batch_window = N >= 16384 ? 16 : 64;
    zeta = smallest_neg_root(t, (uint64_t)N);
    std::vector<uint64_t> pr = find_ntt_primes((uint64_t)N, L + alpha, prime_bits);
    if ((int)pr.size() != L + alpha) throw Error(-1, "not enough primes");
    // the alpha largest are the special primes; extended order q..., p...
    qs.assign(pr.begin() + alpha, pr.end());
    qs.insert(qs.end(), pr.begin(), pr.begin() + alpha);

    kernels_init();

    const int nP = nExt + 1;  // + t
    std::vector<uint64_t> mod(nP);
    for (int r = 0; r < nExt; ++r) mod[r] = qs[r];
    mod[nExt] = t;
    std::vector<double2> qt(nP);
    std::vector<double> twf((size_t)nP * N), twi((size_t)nP * N), ninv(nP);
    for (int r = 0; r < nP; ++r) {
        const uint64_t q = mod[r];
        qt[r] = make_double2((double)q, 1.0 / (double)q);
        const uint64_t psi = (r == nExt) ? zeta : find_psi(q, (uint64_t)N);
        const uint64_t psii = hinv(psi, q);
        for (int i = 0; i < N; ++i) {
            const uint32_t b = bitrev((uint32_t)i, logN);
            twf[(size_t)r * N + i] = centered_d(hpow(psi, b, q), q);
            twi[(size_t)r * N + i] = centered_d(hpow(psii, b, q), q);
        }
        ninv[r] = centered_d(hinv((uint64_t)N % q, q), q);
    }
    // digit lifts
    std::vector<double> mu_invhat(L), mu_hat((size_t)L * nExt);
    for (int i = 0; i < L; ++i) {
        const int j = i / alpha;
        const int d0 = j * alpha, d1 = std::min(d0 + alpha, L);
        uint64_t hat_i = 1;
        for (int s2 = d0; s2 < d1; ++s2)
            if (s2 != i) hat_i = hmul(hat_i, qs[s2] % qs[i], qs[i]);
        mu_invhat[i] = (double)hinv(hat_i, qs[i]);
        for (int r = 0; r < nExt; ++r) {
            uint64_t h = 1;
            for (int s2 = d0; s2 < d1; ++s2)
                if (s2 != i) h = hmul(h, qs[s2] % qs[r], qs[r]);
            mu_hat[(size_t)i * nExt + r] = (double)h;
        }
    }
    // division by P
    std::vector<double> md_coef(alpha), md_hat((size_t)alpha * L), pinv(L);
    for (int k = 0; k < alpha; ++k) {
        const uint64_t pk = qs[L + k];
        uint64_t hat = 1;
        for (int b = 0; b < alpha; ++b)
            if (b != k) hat = hmul(hat, qs[L + b] % pk, pk);
        uint64_t c = hmul(hinv(t % pk, pk), hinv(hat, pk), pk);
        c = hmul(c, hinv((uint64_t)N % pk, pk), pk);
        md_coef[k] = centered_d(c, pk);
        for (int i = 0; i < L; ++i) {
            uint64_t h = 1;
            for (int b = 0; b < alpha; ++b)
                if (b != k) h = hmul(h, qs[L + b] % qs[i], qs[i]);
            md_hat[(size_t)k * L + i] = (double)hmul(t % qs[i], h, qs[i]);
        }
    }
    std::vector<double> pmod(L);
    for (int i = 0; i < L; ++i) {
        uint64_t P = 1;
        for (int k = 0; k < alpha; ++k) P = hmul(P, qs[L + k] % qs[i], qs[i]);
        pinv[i] = centered_d(hinv(P, qs[i]), qs[i]);
        pmod[i] = centered_d(P, qs[i]);
    }
    auto up = [&](const void *src, size_t bytes) -> void * {
        void *p = nullptr;
        HGCHK(hipMalloc(&p, std::max<size_t>(bytes, 256)));
        HGCHK(hipMemcpy(p, src, bytes, hipMemcpyHostToDevice));
        owned.push_back(p);
        return p;
    };
    T.N = N; T.logN = logN; T.L = L; T.alpha = alpha; T.beta = beta; T.nExt = nExt;
    T.qt = (double2 *)up(qt.data(), qt.size() * sizeof(double2));
    T.twf = (double *)up(twf.data(), twf.size() * sizeof(double));
    T.twi = (double *)up(twi.data(), twi.size() * sizeof(double));
    T.ninv = (double *)up(ninv.data(), ninv.size() * sizeof(double));
    T.mu_invhat = (double *)up(mu_invhat.data(), mu_invhat.size() * sizeof(double));
    T.mu_hat = (double *)up(mu_hat.data(), mu_hat.size() * sizeof(double));
    T.md_coef = (double *)up(md_coef.data(), md_coef.size() * sizeof(double));
    T.md_hat = (double *)up(md_hat.data(), md_hat.size() * sizeof(double));
    T.pinv = (double *)up(pinv.data(), pinv.size() * sizeof(double));
    T.pmod = (double *)up(pmod.data(), pmod.size() * sizeof(double));
    T.t = (double)t;
    T.tinv = 1.0 / (double)t;
    // modulus switching from level l to l - 1: P = q_{l-1}, over q_0..q_{l-2}
    ms_tabs.assign(L + 1, DevTables());
    std::vector<double> ms_hat(L);
    for (int i = 0; i < L; ++i) ms_hat[i] = (double)(t % qs[i]);
    double *ms_hat_d = L > 1 ? (double *)up(ms_hat.data(), ms_hat.size() * sizeof(double)) : nullptr;
    for (int l = 2; l <= L; ++l) {
        const uint64_t q = qs[l - 1];
        std::vector<double> coef(1), pinv_l(l - 1);
        coef[0] = centered_d(hmul(hinv(t % q, q), hinv((uint64_t)N % q, q), q), q);
        for (int i = 0; i < l - 1; ++i) pinv_l[i] = centered_d(hinv(q % qs[i], qs[i]), qs[i]);
        DevTables M = T;
        M.L = l - 1;          // output primes
        M.alpha = 1;          // q_{l-1} is the one prime divided out
        M.nExt = l;           // input rows per component
        M.beta = 0;
        M.md_coef = (double *)up(coef.data(), sizeof(double));
        M.md_hat = ms_hat_d;
        M.pinv = (double *)up(pinv_l.data(), pinv_l.size() * sizeof(double));
        M.mu_invhat = M.mu_hat = M.pmod = nullptr;
        ms_tabs[l] = M;
    }
}

Ctx::~Ctx() {
    (void)hipSetDevice(device);
    (void)hipDeviceSynchronize();
    for (auto &kv : arenas) kv.second.release();
    noalloc_arena.release();
    for (auto &kv : aux) {
        for (auto &ring : kv.second.ev)
            for (hipEvent_t e : ring) (void)hipEventDestroy(e);
        if (kv.second.side) (void)hipStreamDestroy(kv.second.side);
    }
    for (auto *v : {&lt_pairs, &lt_md_pairs})
        for (auto &pr : *v) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    for (hipEvent_t e : lt_free) (void)hipEventDestroy(e);
    for (auto &kv : mask_cache) (void)hipFree(kv.second);
    for (auto &kv : rot_keys) (void)hipFree(kv.second);
    if (relin_key) (void)hipFree(relin_key);
    if (s_eval) (void)hipFree(s_eval);
    if (s2_eval) (void)hipFree(s2_eval);
    for (void *p : owned) (void)hipFree(p);
}

double *Ctx::dev_alloc(size_t words) {
    void *p = nullptr;
    HGCHK(hipMalloc(&p, std::max<size_t>(words, 32) * sizeof(double)));
    return (double *)p;
}

hipStream_t Ctx::side_stream(hipStream_t st) {
    StreamAux &a = aux[st];
    if (!a.side) HGCHK(hipStreamCreateWithFlags(&a.side, hipStreamNonBlocking));
    return a.side;
}

hipEvent_t Ctx::event(hipStream_t st, bool timing) {
    // a ring per kind: an event is re-recorded only after 512 others, long
    // after every wait on its earlier record was enqueued and every timing
    // pair read back (a timed call synchronises at its end)
    constexpr size_t RING = 512;
    StreamAux &a = aux[st];
    auto &ring = a.ev[timing ? 1 : 0];
    size_t &nx = a.next[timing ? 1 : 0];
    if (ring.size() < RING) {
        hipEvent_t e;
        HGCHK(hipEventCreateWithFlags(&e, timing ? hipEventDefault : hipEventDisableTiming));
        ring.push_back(e);
        return e;
    }
    hipEvent_t e = ring[nx];
    nx = (nx + 1) % RING;
    return e;
}

hipEvent_t Ctx::lt_event() {
    if (!lt_free.empty()) {
        hipEvent_t e = lt_free.back();
        lt_free.pop_back();
        return e;
    }
    hipEvent_t e;
    HGCHK(hipEventCreate(&e));
    return e;
}

void Arena::release() {
    if (!fixed_bytes) {
        if (base) (void)hipFree(base);
        if (acc) (void)hipFree(acc);
    }
    if (pinned) (void)hipHostFree(pinned);
    if (staged) (void)hipEventDestroy(staged);
    base = pinned = pinned_dev = acc = nullptr;
    staged = nullptr;
    cap = pinned_cap = acc_cap = 0;
    slot = 0;
    copies = 0;
}

Arena &Ctx::arena_for(hipStream_t st) {
    if (fixed_arena) return *fixed_arena;
    if (!capture_arenas) return arena(st);
    auto &v = *capture_arenas;
    if (capture_next == v.size()) {
        if (capturing) throw Error(-5, "graph recording needs a workspace the first pass did not make");
        v.push_back(std::make_unique<Arena>());
        HGCHK(hipEventCreateWithFlags(&v.back()->staged, hipEventDisableTiming));
    }
    return *v[capture_next++];
}

Arena &Ctx::arena(hipStream_t st) {
    Arena &a = arenas[st];
    if (!a.staged) {
        HGCHK(hipEventCreateWithFlags(&a.staged, hipEventDisableTiming));
        a.ring = 8;
    }
    return a;
}

int Ctx::galois_of(int z) const {
    const int zz = ((z % S) + S) % S;
    return galois_tab[zz];
}

const PlanEntry &Ctx::plan_for(int m, int l, int n) {
    auto key = std::make_tuple(m, l, n);
    auto it = plans.find(key);
    if (it != plans.end()) return *it->second;
    auto pe = std::make_unique<PlanEntry>();
    try {
        pe->plan = make_plan(m, l, n, S, method, min_blocks);
    } catch (std::invalid_argument &e) {
        throw Error(-1, e.what());
    } catch (std::range_error &e) {
        throw Error(-2, e.what());
    }
    for (auto &bm : pe->plan.masks) pe->mask_ptrs.push_back(mask_for(bm));
    auto &ref = *pe;
    plans[key] = std::move(pe);
    return ref;
}

// ---------------------------------------------------------------------------
// encoding and masks
// ---------------------------------------------------------------------------

void Ctx::encode_slots(const std::vector<uint64_t> &slots, double *mu, hipStream_t st) {
    std::vector<double> v(S, 0.0);
    for (int s = 0; s < S && s < (int)slots.size(); ++s) v[s] = (double)(slots[s] % t);
    double *ds = dev_alloc(S);
    double *ev = dev_alloc(N);
    HGCHK(hipMemcpyAsync(ds, v.data(), S * sizeof(double), hipMemcpyHostToDevice, st));
    scatter_slots(T, ds, ev, st);
    NttArgs a;
    a.out = mu; a.in = ev; a.rows = 1; a.per = 1; a.prime_base = nExt;
    ntt_inv(T, STORE_PLAIN, a, st);
    center_rows(T, mu, 1, nExt, 1, st);   // the centered lift of mu, exact
    HGCHK(hipStreamSynchronize(st));
    (void)hipFree(ds);
    (void)hipFree(ev);
}

double *Ctx::mask_for(const std::vector<uint8_t> &bitmap) {
    std::string key(bitmap.begin(), bitmap.end());
    auto it = mask_cache.find(key);
    if (it != mask_cache.end()) return it->second;
    std::vector<uint64_t> slots(S);
    for (int s = 0; s < S; ++s) slots[s] = bitmap[s];
    hipStream_t st = nullptr;
    double *mu = dev_alloc(N);
    encode_slots(slots, mu, st);
    double *m = dev_alloc((size_t)nExt * N);
    broadcast_rows(mu, m, N, nExt, st);
    NttArgs a;
    a.out = m; a.in = m; a.rows = nExt; a.per = nExt; a.prime_base = 0;
    a.out_stride = a.in_stride = (long long)nExt * N;
    ntt_fwd(T, LOAD_PLAIN, a, st);
    HGCHK(hipStreamSynchronize(st));
    (void)hipFree(mu);
    mask_cache[key] = m;
    return m;
}

// ---------------------------------------------------------------------------
// keys
// ---------------------------------------------------------------------------

void Ctx::keygen(uint64_t seed_, const std::vector<int> &galois) {
    hipStream_t st = nullptr;
    if (!s_eval) {
        seed = seed_;
        has_secret = true;
        double *s_small = dev_alloc(N);
        sample_small(s_small, stream_state(seed, TAG_SECRET, 0), 0, N, 0, st);
        s_eval = dev_alloc((size_t)nExt * N);
        broadcast_rows(s_small, s_eval, N, nExt, st);
        NttArgs a;
        a.out = s_eval; a.in = s_eval; a.rows = nExt; a.per = nExt;
        a.out_stride = a.in_stride = (long long)nExt * N;
        ntt_fwd(T, LOAD_PLAIN, a, st);
        s2_eval = dev_alloc((size_t)L * N);
        mul_rows(T, s2_eval, s_eval, s_eval, L, 0, L, st);
        HGCHK(hipStreamSynchronize(st));
        (void)hipFree(s_small);
    } else if (seed_ != seed) {
        throw Error(-6, "keys already generated under another seed");
    }
    if (!has_secret) throw Error(-6, "secret key dropped");

    std::vector<double> gad((size_t)beta * nExt, 0.0);
    for (int j = 0; j < beta; ++j) {
        const int d0 = j * alpha, d1 = std::min(d0 + alpha, L);
        for (int r = d0; r < d1; ++r) {
            uint64_t P = 1;
            for (int k = 0; k < alpha; ++k) P = hmul(P, qs[L + k] % qs[r], qs[r]);
            gad[(size_t)j * nExt + r] = (double)P;
        }
    }
    double *dgad = dev_alloc(gad.size());
    HGCHK(hipMemcpy(dgad, gad.data(), gad.size() * sizeof(double), hipMemcpyHostToDevice));
    double *e_small = dev_alloc(N);
    double *e_rows = dev_alloc((size_t)nExt * N);
    double *sp = dev_alloc((size_t)nExt * N);

    // b_j = t e_j - a_j s + [P] s' (the last term on the digit's primes);
    // a_j is the digit stream's uniform draws taken as evaluations (draw
    // r N + i is the value at the i-th evaluation point, natural order), so
    // it is never stored: the key-switching kernels regenerate it.
    auto make_key = [&](uint64_t tag, uint64_t idx_base, const double *sprime) -> double * {
        double *key = dev_alloc(key_words());
        const size_t plane = (size_t)nExt * N;
        std::vector<uint64_t> streams(beta);
        for (int j = 0; j < beta; ++j) {
            const uint64_t s0 = stream_state(seed, tag, idx_base + (uint64_t)j);
            streams[j] = s0;
            double *b = key + (size_t)j * plane;
            sample_small(e_small, s0, (uint64_t)nExt * N, N, 1, st);
            broadcast_rows(e_small, e_rows, N, nExt, st);
            NttArgs na;
            na.rows = nExt; na.per = nExt; na.out_stride = na.in_stride = (long long)plane;
            na.out = e_rows; na.in = e_rows;
            ntt_fwd(T, LOAD_PLAIN, na, st);
            keygen_combine(T, b, s0, e_rows, s_eval, sprime, dgad + (size_t)j * nExt, st);
        }
        key_streams[key] = streams;
        return key;
    };
    if (!relin_key) {
        mul_rows(T, sp, s_eval, s_eval, nExt, 0, nExt, st);   // s^2 in evaluation form
        relin_key = make_key(TAG_RELIN, 0, sp);
    }
    for (int g : galois) {
        if (g == 1 || rot_keys.count(g)) continue;
        automorph_rows(T, sp, s_eval, nExt, g, st);          // phi_g(s)
        rot_keys[g] = make_key(TAG_ROT, (uint64_t)g * 256ULL, sp);
        if (key_of_g.empty()) key_of_g.assign((size_t)2 * N, nullptr);
        key_of_g[g] = rot_keys[g];
    }
    HGCHK(hipStreamSynchronize(st));
    (void)hipFree(dgad);
    (void)hipFree(e_small);
    (void)hipFree(e_rows);
    (void)hipFree(sp);
}

void Ctx::drop_secret() {
    HGCHK(hipDeviceSynchronize());
    has_secret = false;
    // the secret's transform stays only as long as the keys are being made;
    // afterwards encryption and decryption are refused
    if (s_eval) {
        HGCHK(hipMemset(s_eval, 0, (size_t)nExt * N * sizeof(double)));
    }
    if (s2_eval) HGCHK(hipMemset(s2_eval, 0, (size_t)L * N * sizeof(double)));
}

// ---------------------------------------------------------------------------
// encryption / decryption
// ---------------------------------------------------------------------------

Ct *Ctx::encrypt_slots(const std::vector<uint64_t> &slots, int side, int block, uint64_t nonce, Ct *into,
                       int into_index) {
    if (!has_secret) throw Error(-6, "no secret key");
    hipStream_t st = nullptr;
    Ct *c = into;
    if (!c) {
        c = new Ct();
        c->ctx = this;
        c->ncts = 1;
        c->comps = 2;
        ct_alloc(c, st);
    }
    double *c0 = c->ct(into_index);
    double *c1 = c0 + (size_t)L * N;
    const uint64_t s0 = stream_state(seed, TAG_ENC, enc_index(side, block, nonce));
    double *mu = dev_alloc(N);
    encode_slots(slots, mu, st);
    sample_uniform(T, c1, s0, 0, L, 0, st);
    double *e = dev_alloc(N);
    sample_small(e, s0, (uint64_t)L * N, N, 1, st);
    double *noisy = dev_alloc(N);
    enc_noisy(T, noisy, e, mu, st);
    broadcast_rows(noisy, c0, N, L, st);
    NttArgs a;
    a.rows = 2 * L; a.per = L; a.out_stride = a.in_stride = (long long)L * N;
    a.out = c0; a.in = c0;
    ntt_fwd(T, LOAD_PLAIN, a, st);   // both components
    enc_combine(T, c0, c0, c1, s_eval, st);
    HGCHK(hipStreamSynchronize(st));
    (void)hipFree(mu);
    (void)hipFree(e);
    (void)hipFree(noisy);
    return c;
}

Ct *Ctx::encrypt_matrix(int role, const int64_t *X, int m, int l, int n, uint64_t nonce) {
    if (!has_secret) throw Error(-6, "no secret key");
    if (role != 0 && role != 1) throw Error(-1, "role must be 0 (A) or 1 (B)");
    const PlanEntry &pe = plan_for(m, l, n);
    const Plan &p = pe.plan;
    Ct *c = new Ct();
    c->ctx = this;
    c->ncts = p.nb;
    c->comps = 2;
    c->m = m; c->l = l; c->n = n;
    c->side = side_of_role(p, role);
    ct_alloc(c, nullptr);
    try {
        encrypt_matrix_into(role, X, m, l, n, nonce, c, 0);
    } catch (...) {
        delete c;
        throw;
    }
    return c;
}

void Ctx::encrypt_matrix_into(int role, const int64_t *X, int m, int l, int n, uint64_t nonce, Ct *into,
                              int first) {
    const Plan &p = plan_for(m, l, n).plan;
    const int side = side_of_role(p, role);
    for (int b = 0; b < p.nb; ++b) {
        std::vector<uint64_t> v = pack_operand(p, side, X, b, t, S);
        encrypt_slots(v, side, b, nonce, into, first + b);
    }
}

Ct *Ctx::encrypt_blocked(int role, const int64_t *X, int m, int l, int n, uint64_t nonce, const Partition &pt) {
    if (!has_secret) throw Error(-6, "no secret key");
    if (role != 0 && role != 1) throw Error(-1, "role must be 0 (A) or 1 (B)");
    if (nonce >= (1ULL << 47)) throw Error(-1, "nonce of an output-blocked operand must be below 2^47");
    int total = 0;
    for (int mi : pt.rows)
        for (int nj : pt.cols) total += plan_for(mi, l, nj).plan.nb;
    Ct *c = new Ct();
    c->ctx = this;
    c->ncts = total;
    c->comps = 2;
    c->m = m; c->l = l; c->n = n;
    c->side = 10 + role;
    ct_alloc(c, nullptr);
    try {
        int first = 0, k = 0, r0 = 0;
        std::vector<int64_t> sub;
        for (int mi : pt.rows) {
            int c0 = 0;
            for (int nj : pt.cols) {
                // the block's own matrix, row-major: A's rows r0.., or B's columns c0..
                if (role == 0) {
                    sub.assign(X + (size_t)r0 * l, X + (size_t)(r0 + mi) * l);
                } else {
                    sub.resize((size_t)l * nj);
                    for (int r = 0; r < l; ++r)
                        for (int q = 0; q < nj; ++q) sub[(size_t)r * nj + q] = X[(size_t)r * n + c0 + q];
                }
                encrypt_matrix_into(role, sub.data(), mi, l, nj, nonce * 65536 + (uint64_t)k, c, first);
                first += plan_for(mi, l, nj).plan.nb;
                ++k;
                c0 += nj;
            }
            r0 += mi;
        }
    } catch (...) {
        delete c;
        throw;
    }
    return c;
}

bool Ctx::plannable(int m, int l, int n) const {
    try {
        (void)make_plan(m, l, n, S, method, min_blocks);
        return true;
    } catch (std::range_error &) {
        return false;
    }
}

const Ctx::Partition *Ctx::partition_for(int m, int l, int n) {
    if (m <= 0 || l <= 0 || n <= 0) throw Error(-1, "dimensions must be positive");
    auto key = std::make_tuple(m, l, n);
    auto it = partitions.find(key);
    if (it != partitions.end()) return &it->second;
    if (plans.count(key) || plannable(m, l, n)) return nullptr;
    if (method != 2) throw Error(-2, "output blocking needs HEGMM-En (method 2)");
    // the fewest output blocks of near-equal sizes (rows of A, columns of B)
    // whose every block product fits one ciphertext row
    auto split = [](int x, int parts) {
        std::vector<int> v(parts, x / parts);
        for (int i = 0; i < x % parts; ++i) ++v[i];
        return v;
    };
    const long long most = std::min<long long>((long long)m * n, 4096);   // at most 4096 output blocks
    for (long long total = 2; total <= most; ++total)
        for (int br = 1; br <= std::min<long long>(total, m); ++br) {
            if (total % br) continue;
            const int bc = (int)(total / br);
            if (bc > n) continue;
            Partition pt{split(m, br), split(n, bc)};
            bool ok = true;
            for (int mi : {pt.rows.front(), pt.rows.back()})
                for (int nj : {pt.cols.front(), pt.cols.back()}) ok = ok && plannable(mi, l, nj);
            if (!ok) continue;
            return &(partitions[key] = pt);
        }
    throw Error(-2, "no output blocking fits this shape");
}

void Ctx::set_partition(int m, int l, int n, const std::vector<int> &rows, const std::vector<int> &cols) {
    if (m <= 0 || l <= 0 || n <= 0) throw Error(-1, "dimensions must be positive");
    if (method != 2) throw Error(-1, "output blocking needs HEGMM-En (method 2)");
    auto key = std::make_tuple(m, l, n);
    if (plans.count(key)) throw Error(-1, "the shape was already planned as one product");
    int sr = 0, sc = 0;
    for (int r : rows) {
        if (r <= 0) throw Error(-1, "block sizes must be positive");
        sr += r;
    }
    for (int c : cols) {
        if (c <= 0) throw Error(-1, "block sizes must be positive");
        sc += c;
    }
    if (sr != m || sc != n || rows.empty() || cols.empty()) throw Error(-1, "block sizes must add up to m and n");
    if (rows.size() * cols.size() > 4096) throw Error(-1, "at most 4096 output blocks");
    for (int r : rows)
        for (int c : cols)
            if (!plannable(r, l, c)) throw Error(-2, "a block product does not fit one ciphertext");
    partitions[key] = Partition{rows, cols};
}

std::vector<uint64_t> Ctx::to_host_canonical(const double *eval_rows, int rows, hipStream_t st, int per) {
    if (per <= 0) per = L;
    double *tmp = dev_alloc((size_t)rows * N);
    uint64_t *u = nullptr;
    HGCHK(hipMalloc(&u, (size_t)rows * N * sizeof(uint64_t)));
    NttArgs a;
    a.out = tmp; a.in = eval_rows; a.rows = rows; a.per = per; a.out_stride = a.in_stride = (long long)per * N;
    ntt_inv(T, STORE_CANON, a, st);
    dbl_to_u64(tmp, u, (size_t)rows * N, st);
    std::vector<uint64_t> h((size_t)rows * N);
    HGCHK(hipMemcpyAsync(h.data(), u, h.size() * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    HGCHK(hipStreamSynchronize(st));
    (void)hipFree(tmp);
    (void)hipFree(u);
    return h;
}

std::vector<uint64_t> Ctx::decrypt_poly(const Ct &c, int index) {
    if (!has_secret) throw Error(-6, "no secret key");
    hipStream_t st = nullptr;
    // a ciphertext at a lower level (after modulus switching) holds only the
    // first primes of Q: everything below runs over those (L = its level)
    const int L = c.lv();
    DevTables Tl = T;
    Tl.L = L;
    double *v = dev_alloc((size_t)L * N);
    dec_combine(Tl, v, c.ct(index), c.comps, s_eval, s2_eval, st);
    std::vector<uint64_t> res = to_host_canonical(v, L, st, L);
    (void)hipFree(v);
    // Garner mixed-radix reconstruction: x = sum_i a_i R_i, R_i = q_0...q_{i-1}
    std::vector<std::vector<uint64_t>> inv(L, std::vector<uint64_t>(L, 0));
    for (int i = 0; i < L; ++i)
        for (int s2 = 0; s2 < i; ++s2) inv[i][s2] = hinv(qs[s2] % qs[i], qs[i]);
    std::vector<uint64_t> Rt(L);   // R_i mod t
    uint64_t Qt = 1;
    for (int i = 0; i < L; ++i) {
        Rt[i] = Qt;
        Qt = hmul(Qt, qs[i] % t, t);
    }
    // digits of (Q - 1)/2, whose residue mod q_i is (q_i - 1)/2
    auto garner = [&](const uint64_t *vals, uint64_t *dig) {
        for (int i = 0; i < L; ++i) {
            uint64_t x = vals[i] % qs[i];
            for (int s2 = 0; s2 < i; ++s2) x = hmul(hsub(x, dig[s2] % qs[i], qs[i]), inv[i][s2], qs[i]);
            dig[i] = x;
        }
    };
    std::vector<uint64_t> half(L), hd(L);
    for (int i = 0; i < L; ++i) half[i] = (qs[i] - 1) / 2;
    garner(half.data(), hd.data());
    std::vector<uint64_t> out(N), vals(L), dig(L);
    for (int k = 0; k < N; ++k) {
        for (int i = 0; i < L; ++i) vals[i] = res[(size_t)i * N + k];
        garner(vals.data(), dig.data());
        bool above = false;  // x > (Q-1)/2 ?
        for (int i = L - 1; i >= 0; --i) {
            if (dig[i] != hd[i]) { above = dig[i] > hd[i]; break; }
        }
        uint64_t r = 0;
        for (int i = 0; i < L; ++i) r = hadd(r, hmul(dig[i] % t, Rt[i], t), t);
        if (above) r = hsub(r, Qt, t);
        out[k] = r;
    }
    return out;
}

std::vector<uint64_t> Ctx::decrypt_slot_values(const Ct &c, int index) {
    std::vector<uint64_t> mu = decrypt_poly(c, index);
    hipStream_t st = nullptr;
    std::vector<double> md(N);
    for (int i = 0; i < N; ++i) md[i] = (double)mu[i];
    double *dm = dev_alloc(N);
    double *ds = dev_alloc(S);
    HGCHK(hipMemcpyAsync(dm, md.data(), N * sizeof(double), hipMemcpyHostToDevice, st));
    NttArgs a;
    a.out = dm; a.in = dm; a.rows = 1; a.per = 1; a.prime_base = nExt;
    ntt_fwd(T, LOAD_PLAIN, a, st);
    gather_slots(T, dm, ds, st);
    std::vector<double> sv(S);
    HGCHK(hipMemcpyAsync(sv.data(), ds, S * sizeof(double), hipMemcpyDeviceToHost, st));
    HGCHK(hipStreamSynchronize(st));
    (void)hipFree(dm);
    (void)hipFree(ds);
    std::vector<uint64_t> out(S);
    for (int s = 0; s < S; ++s) {
        long long v = (long long)sv[s] % (long long)t;
        out[s] = (uint64_t)(v < 0 ? v + (long long)t : v);
    }
    return out;
}

// ---------------------------------------------------------------------------
// export / import (canonical coefficient form)
// ---------------------------------------------------------------------------

void Ctx::export_ct(const Ct &c, uint64_t *buf, hipStream_t st) {
    const int rows = c.ncts * c.comps * c.lv();
    std::vector<uint64_t> h = to_host_canonical(c.d, rows, st, c.lv());
    std::memcpy(buf, h.data(), h.size() * sizeof(uint64_t));
}

Ct *Ctx::import_ct(const uint64_t *buf, int ncts, int comps, hipStream_t st) {
    Ct *c = new Ct();
    c->ctx = this;
    c->ncts = ncts;
    c->comps = comps;
    ct_alloc(c, st);
    try {
        load_ct(*c, buf, c->words(), st);
    } catch (...) {
        delete c;
        throw;
    }
    return c;
}

void Ctx::load_ct(Ct &c, const uint64_t *buf, size_t nwords, hipStream_t st) {
    const size_t n = c.words();
    const int lv = c.lv();
    if (nwords != n) throw Error(-1, "word count does not match the handle");
    for (size_t r = 0; r < n / N; ++r) {
        const uint64_t q = qs[r % lv];
        for (int i = 0; i < N; ++i)
            if (buf[r * N + i] >= q) throw Error(-1, "residue out of range in import");
    }
    uint64_t *u = nullptr;
    HGCHK(hipMalloc(&u, n * sizeof(uint64_t)));
    HGCHK(hipMemcpyAsync(u, buf, n * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    u64_to_dbl(u, c.d, n, st);
    NttArgs a;
    a.out = c.d; a.in = c.d; a.rows = (int)(n / N); a.per = lv;
    a.out_stride = a.in_stride = (long long)lv * N;
    ntt_fwd(T, LOAD_PLAIN, a, st);
    HGCHK(hipStreamSynchronize(st));
    (void)hipFree(u);
}

}  // namespace hg
