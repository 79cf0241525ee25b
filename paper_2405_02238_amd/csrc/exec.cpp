// Cloud-side executor: HEGMM-En (Algorithm 2) for one or many requests, and
// the single-ciphertext primitives, as a fixed sequence of batched launches.
//
// For a set of "rotation-sum" jobs  T(ct) = sum_z mask_z (.) Rot(ct, z)  the
// executor runs, each phase as one launch over every job of every request:
//   1. hoist: inverse transform of each source c1, digit lift (ModUp) fused
//      into the forward transform of every lifted row;
//   2. inner products of the permuted digits with the rotation keys, masked
//      and summed per job (key-switched terms only);
//   3. division by P: inverse transform of the special-prime rows (storing
//      the centered correction r_k), forward transform of the correction
//      delta over the ciphertext primes;
//   4. finish: masked permuted c0 (and c1 for unrotated terms) plus
//      (U - delta) P^-1, consumed directly by the tensor accumulation.
// Relinearisation (once per product, after the accumulation) and the fold
// of the d row blocks reuse phases 1-4 with a single job per request.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "context.h"

namespace hg {

namespace {

// Host-side description of one phase-1..4 pass.
struct Pass {
    std::vector<const double *> srcs;   // eval-form c1 of each hoisted source (L x N)
    std::vector<IpJob> ip_jobs;         // key-switched jobs
    std::vector<IpTerm> ip_terms;
    std::vector<FinJob> fin_jobs;
    std::vector<FinTerm> fin_terms;
    std::vector<const double *> keys;
    std::unordered_map<const double *, int> key_index;
    std::vector<const double *> masks;
    std::unordered_map<const double *, int> mask_index;

    int key_id(const double *k) {
        auto it = key_index.find(k);
        if (it != key_index.end()) return it->second;
        keys.push_back(k);
        return key_index[k] = (int)keys.size() - 1;
    }
    int mask_id(const double *m) {
        if (!m) return -1;
        auto it = mask_index.find(m);
        if (it != mask_index.end()) return it->second;
        masks.push_back(m);
        return mask_index[m] = (int)masks.size() - 1;
    }
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Byte layout of everything a pass needs in the arena.
struct Layout {
    size_t total = 0;
    size_t add(size_t bytes) {
        size_t off = total;
        total = align_up(total + bytes, 256);
        return off;
    }
};

}  // namespace

namespace {

struct Exec {
    Ctx &C;
    hipStream_t st;
    Arena &A;
    const DevTables &T;
    int N, L, nExt, beta, alpha;
    Exec(Ctx &c, hipStream_t s)
        : C(c), st(s), A(c.arena_for(s)), T(c.T), N(c.N), L(c.L), nExt(c.nExt), beta(c.beta), alpha(c.alpha) {}

    // The staged tables' copy to the device, not yet enqueued: the first
    // launch after stage() either does it in extra workgroups of a fused
    // hoist (sources by value) or enqueues it on its own (flush) before
    // anything reads the tables.
    struct Pending {
        void *dst = nullptr;
        const void *src = nullptr;
        size_t bytes = 0;
        hipEvent_t done = nullptr;   // completion signal the staging ring waits on
    } pend;

    void flush() {
        if (!pend.dst) return;
        copy_from_host(pend.dst, pend.src, pend.bytes, st, pend.done);
        pend = Pending();
    }

    // Accumulator space for this call (stream-ordered reuse of one buffer per
    // arena; grown with the stream drained, never while recording a graph).
    double *acc(size_t bytes) {
        if (A.fixed_bytes) {
            const size_t a = align_up(bytes, 256);
            if (a > A.fixed_bytes)
                throw Error(-1, "the product needs " + std::to_string(a) + " bytes of accumulators; the fixed "
                                "workspace holds " + std::to_string(A.fixed_bytes));
            A.acc = A.fixed_base;
            A.acc_cap = a;
            A.base = A.fixed_base + a;
            A.cap = A.fixed_bytes - a;
            return (double *)A.acc;
        }
        if (bytes > A.acc_cap) {
            if (C.capturing) throw Error(-5, "graph recording needs a workspace the first pass did not make");
            HGCHK(hipStreamSynchronize(st));
            if (A.acc) HGCHK(hipFree(A.acc));
            A.acc_cap = align_up(A.exact ? bytes : bytes + bytes / 4, 1 << 20);
            HGCHK(hipMalloc(&A.acc, A.acc_cap));
        }
        return (double *)A.acc;
    }

    // Adds a job to `ps`: the rotation sum sum_z mask_z (.) Rot(ct, z) over
    // `terms` (z, mask pointer or null), plus the key switch of the hoisted
    // source `src` under relin_key when given.  Jobs that need no key switch
    // are finished from their plain terms.  Returns the job index.
    int add_job(Pass &ps, const double *ct, const std::vector<std::pair<int, const double *>> &terms,
                int src, const double *relin_key) {
        FinJob fj;
        fj.c0 = ct;
        fj.c1 = ct + (size_t)L * N;
        fj.t0 = (int)ps.fin_terms.size();
        fj.nt = 0;
        fj.ks = -1;
        bool ks = relin_key != nullptr;
        int nrot = 0;
        for (auto &tm : terms) nrot += C.galois_of(tm.first) != 1;
        ks |= nrot > 0;
        // The paper's primitive order (ks_order 1): every rotated diagonal is
        // one complete HE-Rot (its own key switch and division by P), then its
        // mask (HE-CMult), then the sum (HE-Add).  A lone unmasked rotation is
        // the same in both orders and stays one job.
        const bool per_rotation =
            C.ks_order == 1 && !relin_key && nrot > 0 && !(terms.size() == 1 && terms[0].second == nullptr);
        if (!ks) {
            for (auto &tm : terms) ps.fin_terms.push_back({1, ps.mask_id(tm.second), -1});
            fj.nt = (int)ps.fin_terms.size() - fj.t0;
        } else if (per_rotation) {
            for (auto &tm : terms) {
                const int g = C.galois_of(tm.first);
                const int mid = ps.mask_id(tm.second);
                if (g == 1) {
                    ps.fin_terms.push_back({1, mid, -1});
                    continue;
                }
                const double *key = C.rot_key(g);
                if (!key) throw Error(-3, "missing rotation key for z = " + std::to_string(tm.first));
                IpJob ij;
                ij.c0 = fj.c0;
                ij.c1 = fj.c1;
                ij.src = src;
                ij.t0 = (int)ps.ip_terms.size();
                ij.nt = 1;
                ij.slot = (int)ps.ip_jobs.size();
                ps.ip_terms.push_back({g, -1, ps.key_id(key), IP_ROT});
                ps.fin_terms.push_back({1, mid, ij.slot});
                ps.ip_jobs.push_back(ij);
            }
            fj.nt = (int)ps.fin_terms.size() - fj.t0;
        } else {
            IpJob ij;
            ij.c0 = fj.c0;
            ij.c1 = fj.c1;
            ij.src = src;
            ij.t0 = (int)ps.ip_terms.size();
            ij.slot = (int)ps.ip_jobs.size();
            for (auto &tm : terms) {
                const int g = C.galois_of(tm.first);
                const int mid = ps.mask_id(tm.second);
                if (g == 1) {
                    ps.ip_terms.push_back({1, mid, -1, IP_PLAIN});
                } else {
                    const double *key = C.rot_key(g);
                    if (!key) throw Error(-3, "missing rotation key for z = " + std::to_string(tm.first));
                    ps.ip_terms.push_back({g, mid, ps.key_id(key), IP_ROT});
                }
            }
            if (relin_key) ps.ip_terms.push_back({1, -1, ps.key_id(relin_key), IP_RELIN});
            ij.nt = (int)ps.ip_terms.size() - ij.t0;
            fj.ks = (int)ps.ip_jobs.size();
            ps.ip_jobs.push_back(ij);
        }
        ps.fin_jobs.push_back(fj);
        return (int)ps.fin_jobs.size() - 1;
    }

    // Device views of a staged pass.
    struct Dev {
        double *U = nullptr, *E = nullptr;
        FinJob *jobs = nullptr;
        FinTerm *terms = nullptr;
        const double *const *masks = nullptr;
        char *extra = nullptr;   // caller-requested table space
        // internal
        char *tab = nullptr;
        size_t t_ipj = 0, t_ipt = 0, t_keys = 0, t_streams = 0, t_srcs = 0, t_chunks = 0, t_tasks = 0;
        int nchunks = 0;          // > 0: key-stationary inner products
        std::vector<int> rounds;  // first chunk of each round, then the chunk count
        double *coef = nullptr, *y = nullptr, *rk = nullptr;
        int nsrc = 0, nks = 0;
        const std::vector<const double *> *srcs_h = nullptr;   // the hoisted sources (host copy of the table)
        // the pass's key-switched terms use each key at least twice on
        // average: its inner products read keys and masks through the caches
        bool key_reuse = false;
        // one job of at most two terms whose key switches share one key (a
        // relinearisation, a single rotation): its inner products take the
        // job, terms, key and streams by value (ip_one_launch)
        bool one_ok = false;
        IpOne one{};
    };

    struct Staged {
        Pass *ps;
        const void *extra;
        size_t extra_bytes;
        Dev dv;
    };

    // Key-stationary schedule of a pass's key-switched terms: round s takes
    // the s-th key-switched term of every job that has one; within a round,
    // tasks (job, term) with the same key form chunks of at most ip_chunk.
    // rounds[s] is the first chunk of round s (rounds.back() = chunk count).
    // Returns false (one plain launch) when key grouping is off or keys would
    // be used fewer than four times on average (below that, gathering the
    // hoisted digits of many products costs more than the key reads saved;
    // measured on MI355X with groups of four 16384-point products).
    bool group_jobs(const Pass &ps, std::vector<int2> &chunks, std::vector<int2> &tasks, std::vector<int> &rounds) {
        const int nj = (int)ps.ip_jobs.size();
        if (C.ip_chunk <= 0 || nj < 2) return false;
        std::vector<std::map<int, std::vector<int2>>> by_round;   // round -> key -> tasks
        for (int j = 0; j < nj; ++j) {
            const IpJob &J = ps.ip_jobs[j];
            int s = 0;
            for (int t = J.t0; t < J.t0 + J.nt; ++t) {
                const IpTerm &tm = ps.ip_terms[t];
                if (tm.kind == IP_PLAIN) continue;
                if ((int)by_round.size() <= s) by_round.emplace_back();
                by_round[s][tm.key].push_back(make_int2(j, t));
                ++s;
            }
        }
        size_t groups = 0, ntask = 0;
        for (auto &rd : by_round) {
            groups += rd.size();
            for (auto &kv : rd) ntask += kv.second.size();
        }
        if (groups * 4 > ntask) return false;   // keys used fewer than four times on average
        for (auto &rd : by_round) {
            rounds.push_back((int)chunks.size());
            for (auto &kv : rd) {
                const auto &v = kv.second;
                for (size_t o = 0; o < v.size(); o += C.ip_chunk) {
                    const int cnt = (int)std::min<size_t>(C.ip_chunk, v.size() - o);
                    chunks.push_back(make_int2((int)tasks.size(), cnt));
                    tasks.insert(tasks.end(), v.begin() + o, v.begin() + o + cnt);
                }
            }
        }
        rounds.push_back((int)chunks.size());
        return true;
    }

    // The pass's jobs ordered by the keys of their key-switched terms
    // (stable: ties keep their order).
    static std::vector<IpJob> key_order(const Pass &ps) {
        std::vector<std::pair<std::vector<int>, int>> ks(ps.ip_jobs.size());
        for (size_t j = 0; j < ps.ip_jobs.size(); ++j) {
            const IpJob &J = ps.ip_jobs[j];
            for (int t = J.t0; t < J.t0 + J.nt; ++t)
                if (ps.ip_terms[t].kind != IP_PLAIN) ks[j].first.push_back(ps.ip_terms[t].key);
            ks[j].second = (int)j;
        }
        std::stable_sort(ks.begin(), ks.end());
        std::vector<IpJob> out;
        out.reserve(ks.size());
        for (auto &k : ks) out.push_back(ps.ip_jobs[k.second]);
        return out;
    }

    // Lay out the scratch of several passes that run one after another on
    // the stream (one scratch region sized for the largest, one descriptor
    // table block per pass) and copy every table with a single transfer.
    void stage(std::vector<Staged> &sp) {
        size_t scratch = 0;
        std::vector<size_t> toff(sp.size());
        Layout tl;
        struct Off { size_t ipj, ipt, fj, ft, keys, streams, masks, extra, srcs, chunks, jlist; };
        std::vector<std::vector<uint64_t>> streams(sp.size());
        for (size_t i = 0; i < sp.size(); ++i)
            for (const double *k : sp[i].ps->keys) {
                const auto &ks = C.key_streams.at(k);
                streams[i].insert(streams[i].end(), ks.begin(), ks.end());
            }
        std::vector<Off> off(sp.size());
        std::vector<std::vector<int2>> chunks(sp.size());
        std::vector<std::vector<int2>> tasks(sp.size());
        std::vector<std::vector<int>> rounds(sp.size());
        for (size_t i = 0; i < sp.size(); ++i)
            if (!group_jobs(*sp[i].ps, chunks[i], tasks[i], rounds[i])) {
                chunks[i].clear();
                tasks[i].clear();
                rounds[i].clear();
            }
        for (size_t i = 0; i < sp.size(); ++i) {
            Pass &ps = *sp[i].ps;
            const size_t nsrc = ps.srcs.size(), nks = ps.ip_jobs.size();
            Layout lay;
            lay.add(nsrc * L * N * 8);
            lay.add(nsrc * beta * nExt * N * 8);
            lay.add(nks * 2 * nExt * N * 8);
            lay.add(nks * 2 * alpha * N * 8);
            lay.add(nks * 2 * L * N * 8);
            scratch = std::max(scratch, lay.total);
            Off &o = off[i];
            o.ipj = tl.add(ps.ip_jobs.size() * sizeof(IpJob));
            o.ipt = tl.add(ps.ip_terms.size() * sizeof(IpTerm));
            o.fj = tl.add(ps.fin_jobs.size() * sizeof(FinJob));
            o.ft = tl.add(ps.fin_terms.size() * sizeof(FinTerm));
            o.keys = tl.add(ps.keys.size() * sizeof(void *));
            o.streams = tl.add(streams[i].size() * sizeof(uint64_t));
            o.masks = tl.add(ps.masks.size() * sizeof(void *));
            o.extra = tl.add(sp[i].extra_bytes);
            o.srcs = tl.add(ps.srcs.size() * sizeof(void *));
            o.chunks = tl.add(chunks[i].size() * sizeof(int2));
            o.jlist = tl.add(tasks[i].size() * sizeof(int2));
        }
        tl.add(256);   // never empty
        const size_t total = scratch + tl.total;
        if (A.fixed_bytes && (total > A.cap || tl.total > A.pinned_cap))
            throw Error(-1, "the product needs " + std::to_string(total + (A.fixed_bytes - A.cap)) +
                                " bytes of workspace (" + std::to_string(tl.total) + " of descriptor tables); the "
                                "fixed workspace holds " + std::to_string(A.fixed_bytes) + " (" +
                                std::to_string(A.pinned_cap) + " of tables)");
        if ((total > A.cap || tl.total > A.pinned_cap) && C.capturing)
            throw Error(-5, "graph recording needs a workspace the first pass did not make");
        if (total > A.cap) {
            HGCHK(hipStreamSynchronize(st));
            if (A.base) HGCHK(hipFree(A.base));
            A.cap = align_up(A.exact ? total : total + total / 4, 1 << 20);
            HGCHK(hipMalloc(&A.base, A.cap));
        }
        const bool ringed = A.ring > 1;
        if (tl.total > A.pinned_cap) {
            // every copy out of the old staging is done (a ring's last
            // signal need not cover the latest copies: drain its stream)
            if (ringed) HGCHK(hipStreamSynchronize(st));
            else HGCHK(hipEventSynchronize(A.staged));
            if (A.pinned) HGCHK(hipHostFree(A.pinned));
            A.pinned_cap = align_up(tl.total * 2, 1 << 16);
            HGCHK(hipHostMalloc(&A.pinned, A.pinned_cap * (size_t)A.ring, hipHostMallocDefault));
            HGCHK(hipHostGetDevicePointer(&A.pinned_dev, A.pinned, 0));
            A.slot = 0;
            A.copies = 0;
        }
        // the previous copy out of the slot about to be written is done: one
        // slot, the last copy; a ring, on entering its first slot again, the
        // copy out of its last slot and so every earlier one on the stream
        // (a graph's arenas are private and were drained before recording)
        if (!C.capturing && (!ringed || (A.slot == 0 && A.copies >= (uint64_t)A.ring)))
            HGCHK(hipEventSynchronize(A.staged));
        char *h = (char *)A.pinned + (size_t)A.slot * A.pinned_cap;
        const char *h_dev = (const char *)A.pinned_dev + (size_t)A.slot * A.pinned_cap;
        char *base = (char *)A.base;
        char *tab = base + scratch;
        auto put = [&](size_t o, const void *src, size_t bytes) {
            if (bytes) std::memcpy(h + o, src, bytes);
        };
        for (size_t i = 0; i < sp.size(); ++i) {
            Pass &ps = *sp[i].ps;
            const Off &o = off[i];
            if (chunks[i].empty() && C.ip_order && C.pipeline <= 1) {
                // one plain launch: jobs ordered by their key sequence, so that
                // jobs reading the same keys run side by side and find them in
                // cache (bit-neutral: each job writes its own slot)
                const std::vector<IpJob> sorted = key_order(ps);
                put(o.ipj, sorted.data(), sorted.size() * sizeof(IpJob));
            } else {
                put(o.ipj, ps.ip_jobs.data(), ps.ip_jobs.size() * sizeof(IpJob));
            }
            put(o.ipt, ps.ip_terms.data(), ps.ip_terms.size() * sizeof(IpTerm));
            put(o.fj, ps.fin_jobs.data(), ps.fin_jobs.size() * sizeof(FinJob));
            put(o.ft, ps.fin_terms.data(), ps.fin_terms.size() * sizeof(FinTerm));
            put(o.keys, ps.keys.data(), ps.keys.size() * sizeof(void *));
            put(o.streams, streams[i].data(), streams[i].size() * sizeof(uint64_t));
            put(o.masks, ps.masks.data(), ps.masks.size() * sizeof(void *));
            put(o.extra, sp[i].extra, sp[i].extra_bytes);
            put(o.srcs, ps.srcs.data(), ps.srcs.size() * sizeof(void *));
            put(o.chunks, chunks[i].data(), chunks[i].size() * sizeof(int2));
            put(o.jlist, tasks[i].data(), tasks[i].size() * sizeof(int2));
            Dev &dv = sp[i].dv;
            dv.t_chunks = o.chunks;
            dv.t_tasks = o.jlist;
            dv.nchunks = (int)chunks[i].size();
            dv.rounds = rounds[i];
            dv.tab = tab;
            dv.jobs = (FinJob *)(tab + o.fj);
            dv.terms = (FinTerm *)(tab + o.ft);
            dv.masks = (const double *const *)(tab + o.masks);
            dv.extra = tab + o.extra;
            dv.t_ipj = o.ipj;
            dv.t_ipt = o.ipt;
            dv.t_keys = o.keys;
            dv.t_streams = o.streams;
            dv.t_srcs = o.srcs;
            dv.nsrc = (int)ps.srcs.size();
            dv.srcs_h = &ps.srcs;
            dv.nks = (int)ps.ip_jobs.size();
            size_t switched = 0;
            for (const IpTerm &tm : ps.ip_terms) switched += tm.kind != IP_PLAIN;
            dv.key_reuse = switched >= 2 * ps.keys.size() && !ps.keys.empty();
            dv.one_ok = false;
            if (ps.ip_jobs.size() == 1 && ps.ip_jobs[0].nt >= 1 && ps.ip_jobs[0].nt <= IP_ONE_MAX_TERMS &&
                beta <= IP_ONE_MAX_BETA) {
                const IpJob &J = ps.ip_jobs[0];
                dv.one = IpOne{};
                dv.one.J = J;
                int key = -1;
                bool ok = true;
                for (int u = 0; u < J.nt; ++u) {
                    const IpTerm &tm = ps.ip_terms[J.t0 + u];
                    dv.one.tm[u] = tm;
                    dv.one.mask[u] = tm.mask >= 0 ? ps.masks[tm.mask] : nullptr;
                    if (tm.kind != IP_PLAIN) {
                        ok = ok && tm.key >= 0 && (key < 0 || key == tm.key);
                        key = tm.key;
                    }
                }
                if (key >= 0) {
                    dv.one.key = ps.keys[key];
                    for (int j = 0; j < beta; ++j) dv.one.st[j] = streams[i][(size_t)key * beta + j];
                }
                dv.one_ok = ok;
            }
            Layout lay;
            dv.coef = (double *)(base + lay.add((size_t)dv.nsrc * L * N * 8));
            dv.y = (double *)(base + lay.add((size_t)dv.nsrc * beta * nExt * N * 8));
            dv.U = (double *)(base + lay.add((size_t)dv.nks * 2 * nExt * N * 8));
            dv.rk = (double *)(base + lay.add((size_t)dv.nks * 2 * alpha * N * 8));
            dv.E = (double *)(base + lay.add((size_t)dv.nks * 2 * L * N * 8));
        }
        // a kernel reads the tables straight out of the pinned buffer: cheaper
        // on the stream than a copy-engine transfer and its barrier
        const bool signal = !C.capturing && (!ringed || A.slot == A.ring - 1);
        flush();   // a previous stage's copy (not expected: every stage is launched)
        pend.dst = tab;
        pend.src = h_dev;
        pend.bytes = tl.total;
        pend.done = signal ? A.staged : nullptr;
        if (ringed) {
            A.slot = (A.slot + 1) % A.ring;
            ++A.copies;
        }
    }

    // True when a pass's result per job is exactly its division by P (every
    // job key-switched, job j's output is E slot pair j): the fused division
    // can then write the job outputs itself.
    static bool direct_ok(const Pass &ps) {
        if (ps.fin_jobs.size() != ps.ip_jobs.size()) return false;
        for (size_t j = 0; j < ps.fin_jobs.size(); ++j)
            if (ps.fin_jobs[j].ks != (int)j) return false;
        return true;
    }

    // Division by P of the key-switched jobs [j0, j1) of a staged pass; with
    // `outs` (fused only) the results go straight to the jobs' outputs.
    void moddown(const Dev &dv, int j0, int j1, bool fuse, hipStream_t s, double *const *outs = nullptr,
                 Timing *tm = nullptr) {
        const int nj = j1 - j0;
        if (nj <= 0) return;
        double *U = dv.U + (size_t)j0 * 2 * nExt * N;
        double *E = dv.E + (size_t)j0 * 2 * L * N;
        if (fuse) {
            moddown_fused(T, E, U, nj * 2, s, outs ? outs + j0 : nullptr);
            return;
        }
        double *rk = dv.rk + (size_t)j0 * 2 * alpha * N;
        // few rows: each inverse row on two workgroups (input halves), its
        // last stage done by the forward transform's load step
        const int halves = ntt_halves_ok(T, nj * 2 * alpha) ? 1 : 0;
        NttArgs md;
        md.halves = halves;
        md.out = rk;
        md.in = U;
        md.rows = nj * 2 * alpha;
        md.per = alpha;
        md.prime_base = L;
        md.out_stride = (long long)alpha * N;
        md.in_stride = (long long)nExt * N;
        md.in_offset = (long long)L * N;
        ntt_inv(T, STORE_MDR, md, s);
        NttArgs dl;
        dl.halves = halves;
        dl.out = E;
        dl.in = rk;
        dl.aux = U;
        dl.rows = nj * 2 * L;
        dl.in_stride = (long long)alpha * N;
        hipEvent_t t0 = nullptr, t1 = nullptr;
        if (tm) {
            t0 = tm->pooled ? C.lt_event() : C.event(s, true);
            t1 = tm->pooled ? C.lt_event() : C.event(s, true);
            tm->md_pairs.push_back({t0, t1});
        }
        ntt_fwd(T, LOAD_DELTA, dl, s, t0, t1);
    }

    // Phases 1-3 of a staged pass: hoist, inner products, division by P.
    // With C.pipeline > 1 the key-switched jobs run in that many chunks: the
    // inner products of chunk c+1 (bandwidth bound) overlap the division by
    // P of chunk c (transform bound) on a second stream; `st` then waits for
    // the last division.  Timing events (tev) bracket the phases on `st`;
    // ip_ms accumulates the duration of each inner-product launch.
    // Returns true when the division by P wrote the job outputs (`direct`
    // given and the fused path taken): no finishing kernel is needed then.
    bool launch(const Dev &dv, hipEvent_t *tev = nullptr, bool transform_pass = false, Timing *tm = nullptr,
                double *const *direct = nullptr) {
        // few rows: one fused launch per chain (latency bound); many rows:
        // separate launches (throughput bound)
        const bool fuse_hoist = fused_ok(T) && dv.nsrc * beta * nExt <= C.fuse_rows;
        if (dv.nks > 0 && fuse_hoist) {
            if (pend.dst && dv.srcs_h && (int)dv.srcs_h->size() == dv.nsrc && hoist_copy_ok(dv.nsrc, pend.bytes)) {
                // the first launch of the call: the hoist takes its sources
                // by value and copies the tables in extra workgroups
                HoistSrc a{};
                for (int i = 0; i < dv.nsrc; ++i) a.p[i] = (*dv.srcs_h)[i];
                a.copy_src = (const uint4 *)pend.src;
                a.copy_dst = (uint4 *)pend.dst;
                a.copy_n = pend.bytes / 16;
                a.copy_wgs = (int)std::min<size_t>(8, (a.copy_n + 1023) / 1024);
                hoist_fused_copy(T, dv.y, a, dv.nsrc, st, pend.done);
                pend = Pending();
            } else if (dv.srcs_h && (int)dv.srcs_h->size() == dv.nsrc && dv.nsrc <= HOIST_MAX_SRC) {
                flush();
                HoistSrc a{};
                for (int i = 0; i < dv.nsrc; ++i) a.p[i] = (*dv.srcs_h)[i];
                hoist_fused_v(T, dv.y, a, dv.nsrc, st);
            } else {
                flush();
                hoist_fused(T, dv.y, (const double *const *)(dv.tab + dv.t_srcs), dv.nsrc, st);
            }
        }
        flush();
        if (dv.nks <= 0) {
            if (tev)
                for (int i = 0; i < 3; ++i) HGCHK(hipEventRecord(tev[i], st));
            return false;
        }
        if (!fuse_hoist) {
            // 1. hoist every source once: c1 -> coefficient form -> lifted digits
            NttArgs a;
            a.out = dv.coef;
            a.in_tab = (const double *const *)(dv.tab + dv.t_srcs);
            a.rows = dv.nsrc * L;
            a.per = L;
            a.out_stride = (long long)L * N;
            ntt_inv(T, STORE_PLAIN, a, st);
            NttArgs mu;
            mu.out = dv.y;
            mu.in = dv.coef;
            mu.rows = dv.nsrc * beta * nExt;
            mu.in_stride = (long long)L * N;
            ntt_fwd(T, LOAD_MODUP, mu, st);
        }
        if (tev) HGCHK(hipEventRecord(tev[0], st));
        const double *const *keys = (const double *const *)(dv.tab + dv.t_keys);
        const uint64_t *streams = (const uint64_t *)(dv.tab + dv.t_streams);
        const IpJob *jobs = (const IpJob *)(dv.tab + dv.t_ipj);
        const IpTerm *terms = (const IpTerm *)(dv.tab + dv.t_ipt);
        // 2. inner products
        if (dv.nchunks > 0) {
            const int2 *chunks = (const int2 *)(dv.tab + dv.t_chunks);
            for (size_t s = 0; s + 1 < dv.rounds.size(); ++s) {
                hipEvent_t t0 = nullptr, t1 = nullptr;
                if (tm) {
                    t0 = tm->pooled ? C.lt_event() : C.event(st, true);
                    t1 = tm->pooled ? C.lt_event() : C.event(st, true);
                }
                ip_keyed_launch(T, dv.U, dv.y, keys, streams, dv.masks, jobs, terms, chunks + dv.rounds[s],
                                (const int2 *)(dv.tab + dv.t_tasks), dv.rounds[s + 1] - dv.rounds[s], s == 0,
                                transform_pass, st, t0, t1);
                if (tm) tm->ip_pairs.push_back({t0, t1});
            }
            if (tev) HGCHK(hipEventRecord(tev[1], st));
            const bool fz = fused_ok(T) && dv.nks * 2 * L <= C.fuse_rows;
            moddown(dv, 0, dv.nks, fz, st, fz ? direct : nullptr);
            if (tev) HGCHK(hipEventRecord(tev[2], st));
            return fz && direct;
        }
        const int nch = C.capturing ? 1 : std::max(1, std::min(C.pipeline, dv.nks));
        // a chunk's division by P is fused when the chunk is small enough
        const int per_chunk = (dv.nks + nch - 1) / nch;
        const bool fuse_md = fused_ok(T) && per_chunk * 2 * L <= C.fuse_rows;
        hipStream_t s2 = nch > 1 ? C.side_stream(st) : st;
        for (int c = 0; c < nch; ++c) {
            const int j0 = (int)((long long)dv.nks * c / nch), j1 = (int)((long long)dv.nks * (c + 1) / nch);
            hipEvent_t t0 = nullptr, t1 = nullptr;
            if (tm) {
                t0 = tm->pooled ? C.lt_event() : C.event(st, true);
                t1 = tm->pooled ? C.lt_event() : C.event(st, true);
            }
            if (dv.one_ok && nch == 1)
                ip_one_launch(T, dv.U, dv.y, dv.one, st, t0, t1);
            else
                ip_launch(T, dv.U, dv.y, keys, streams, dv.masks, jobs + j0, terms, j1 - j0, transform_pass, st, t0,
                          t1, dv.key_reuse);
            if (tm) tm->ip_pairs.push_back({t0, t1});
            if (tev && c == nch - 1) HGCHK(hipEventRecord(tev[1], st));
            if (s2 != st) {
                hipEvent_t ev = C.event(st, false);
                HGCHK(hipEventRecord(ev, st));
                HGCHK(hipStreamWaitEvent(s2, ev, 0));
            }
            moddown(dv, j0, j1, fuse_md, s2, fuse_md ? direct : nullptr, tm);
        }
        if (s2 != st) {
            hipEvent_t ev = C.event(st, false);
            HGCHK(hipEventRecord(ev, s2));
            HGCHK(hipStreamWaitEvent(st, ev, 0));
        }
        if (tev) HGCHK(hipEventRecord(tev[2], st));
        return fuse_md && direct;
    }

    // Stage and launch a single pass.
    Dev run(Pass &ps, const void *extra_host, size_t extra_bytes, hipEvent_t *tev = nullptr) {
        std::vector<Staged> sp{{&ps, extra_host, extra_bytes, Dev()}};
        stage(sp);
        launch(sp[0].dv, tev);
        return sp[0].dv;
    }
};

}  // namespace

Graph::Graph(Ctx &c, std::vector<Ctx::Request> &reqs) : C(&c) {
    HGCHK(hipSetDevice(c.device));
    HGCHK(hipStreamCreateWithFlags(&gs, hipStreamNonBlocking));
    // neither timing mode applies to the recorded launches
    const bool timing = c.timing.enabled, launch_timing = c.launch_timing;
    c.timing.enabled = false;
    c.launch_timing = false;
    c.capture_arenas = &arenas;
    c.capture_next = 0;
    bool recording = false;
    try {
        // a first, eager pass makes and sizes every workspace and descriptor
        // table, so that the recorded pass neither allocates nor waits
        c.hegmm_batch(reqs, gs);
        HGCHK(hipStreamSynchronize(gs));
        c.capture_next = 0;
        c.capturing = true;
        HGCHK(hipStreamBeginCapture(gs, hipStreamCaptureModeRelaxed));
        recording = true;
        c.hegmm_batch(reqs, gs);
        recording = false;
        HGCHK(hipStreamEndCapture(gs, &g));
        HGCHK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
    } catch (...) {
        if (recording) {
            hipGraph_t tmp = nullptr;
            (void)hipStreamEndCapture(gs, &tmp);
            if (tmp) (void)hipGraphDestroy(tmp);
        }
        c.capturing = false;
        c.capture_arenas = nullptr;
        c.timing.enabled = timing;
        c.launch_timing = launch_timing;
        (void)hipStreamSynchronize(gs);
        for (auto &a : arenas) a->release();
        (void)hipStreamDestroy(gs);
        gs = nullptr;
        throw;
    }
    c.capturing = false;
    c.capture_arenas = nullptr;
    c.timing.enabled = timing;
    c.launch_timing = launch_timing;
}

void Graph::launch(hipStream_t st) {
    HGCHK(hipSetDevice(C->device));
    HGCHK(hipGraphLaunch(ge, st));
}

Graph::~Graph() {
    if (!C) return;
    (void)hipSetDevice(C->device);
    (void)hipDeviceSynchronize();
    if (ge) (void)hipGraphExecDestroy(ge);
    if (g) (void)hipGraphDestroy(g);
    for (auto &a : arenas) a->release();
    if (gs) (void)hipStreamDestroy(gs);
}

const PlanEntry &Ctx::check_request(const Request &r) {
    if (!r.A || !r.B) throw Error(-1, "null operand");
    const PlanEntry &pe = plan_for(r.m, r.l, r.n);
    const Ct *A = r.A, *B = r.B;
    if (A->m != r.m || A->l != r.l || A->n != r.n || B->m != r.m || B->l != r.l || B->n != r.n)
        throw Error(-1, "operand shape differs from (m, l, n)");
    if (A->side != side_of_role(pe.plan, 0) || B->side != side_of_role(pe.plan, 1))
        throw Error(-1, "operands must be hg_encrypt outputs for roles 0 (A) and 1 (B)");
    if (A->ncts != pe.plan.nb || B->ncts != pe.plan.nb) throw Error(-1, "block count mismatch");
    need_full_level(*A);
    need_full_level(*B);
    if (!pe.keys_found.load(std::memory_order_relaxed)) {
        for (auto &rz : pe.plan.rotations(S))
            if (!rot_key(galois_of(rz))) throw Error(-3, "missing rotation key for z = " + std::to_string(rz));
        pe.keys_found.store(true, std::memory_order_relaxed);
    }
    return pe;
}

void Ctx::hegmm_batch(std::vector<Request> &reqs, hipStream_t st) {
    HGCHK(hipSetDevice(device));
    // every request is checked before any launch, so an error leaves no
    // work of this call on the stream
    for (auto &r : reqs) check_request(r);
    if (batch_window > 0 && (int)reqs.size() > batch_window) {
        for (size_t o = 0; o < reqs.size(); o += batch_window) {
            std::vector<Request> part(reqs.begin() + o,
                                      reqs.begin() + std::min(reqs.size(), o + (size_t)batch_window));
            hegmm_batch_window(part, st);
        }
        return;
    }
    hegmm_batch_window(reqs, st);
}

void Ctx::hegmm_batch_window(std::vector<Request> &reqs, hipStream_t st) {
    Exec ex(*this, st);
    const size_t ctw = (size_t)L * N;
    // --- validate and plan ---
    struct RInfo {
        const PlanEntry *pe;
        const Ct *X;
        const Ct *Y;
    };
    std::vector<RInfo> info;
    for (auto &r : reqs) {
        const PlanEntry &pe = check_request(r);
        const Ct *X = r.A->side == 0 ? r.A : r.B;
        const Ct *Y = r.A->side == 0 ? r.B : r.A;
        info.push_back({&pe, X, Y});
    }
    const int nreq = (int)reqs.size();
    hipEvent_t ev[10] = {nullptr};
    if (timing.enabled) {
        for (auto &e : ev) HGCHK(hipEventCreate(&e));
        HGCHK(hipEventRecord(ev[9], st));
    }

    // request-lifetime buffers: accumulators (3 x L x N) and relinearised R
    // (2 x L x N, fold only).  Eager relinearisation keeps every loop product
    // apart instead: one three-component tensor per (eps, omega) pair, then
    // its relinearised two-component ciphertext, summed per request after the
    // key switches.  Algorithm 1 with sigma / tau in the cloud (method 3)
    // keeps sigma(X) and tau(Y) of each such request.
    const bool eager = relin == 1;
    int nfold = 0, nst = 0, npairs = 0;
    for (int ri = 0; ri < nreq; ++ri) {
        const Plan &p = info[ri].pe->plan;
        nfold += p.d > 1;
        nst += p.method == 3;
        npairs += p.nb * p.K;
    }
    const int nacc = eager ? npairs : nreq;
    double *acc = ex.acc(((size_t)nacc * 3 + (size_t)nfold * 2 + (eager ? (size_t)npairs * 2 : 0) +
                          (size_t)nst * 4) * ctw * sizeof(double));
    double *rbuf = acc + (size_t)nacc * 3 * ctw;
    double *ebuf = rbuf + (size_t)nfold * 2 * ctw;                  // eager: relinearised products
    double *sbuf = ebuf + (eager ? (size_t)npairs * 2 * ctw : 0);   // method 3: sigma(X), tau(Y)

    // --- method 3: sigma(X) and tau(Y) as rotation sums (Theorems 1 and 2) ---
    Pass pst;
    std::vector<double *> st_out;   // the pass's job outputs
    std::vector<const double *> opX(nreq, nullptr), opY(nreq, nullptr);
    for (int ri = 0, si = 0; ri < nreq; ++ri) {
        const Plan &p = info[ri].pe->plan;
        if (p.method != 3) continue;
        const auto &mp = info[ri].pe->mask_ptrs;
        double *xs = sbuf + (size_t)(si++) * 4 * ctw, *ys = xs + 2 * ctw;
        auto add = [&](const std::vector<Term> &tms, const double *in, double *out) {
            std::vector<std::pair<int, const double *>> te;
            bool k = false;
            for (auto &tm : tms) {
                te.push_back({tm.z, tm.mask >= 0 ? mp[tm.mask] : nullptr});
                k |= galois_of(tm.z) != 1;
            }
            int src = -1;
            if (k) {
                src = (int)pst.srcs.size();
                pst.srcs.push_back(in + ctw);
            }
            ex.add_job(pst, in, te, src, nullptr);
            st_out.push_back(out);
        };
        add(p.sigma, info[ri].X->ct(0), xs);
        add(p.tau, info[ri].Y->ct(0), ys);
        opX[ri] = xs;
        opY[ri] = ys;
    }

    // --- main pass: every eps^k / omega^k transform, then tensor accumulation ---
    Pass ps;
    std::vector<int2> req_pairs(nreq);
    for (int ri = 0; ri < nreq; ++ri) {
        const Plan &p = info[ri].pe->plan;
        const auto &mp = info[ri].pe->mask_ptrs;
        req_pairs[ri] = make_int2((int)ps.fin_jobs.size() / 2, p.nb * p.K);
        for (int b = 0; b < p.nb; ++b) {
            const double *xc = opX[ri] ? opX[ri] : info[ri].X->ct(b);
            const double *yc = opY[ri] ? opY[ri] : info[ri].Y->ct(b);
            int sx = -1, sy = -1;
            for (int k = 0; k < p.K; ++k) {
                std::vector<std::pair<int, const double *>> te, tw;
                bool kx = false, ky = false;
                for (auto &tm : p.eps[k]) {
                    te.push_back({tm.z, tm.mask >= 0 ? mp[tm.mask] : nullptr});
                    kx |= galois_of(tm.z) != 1;
                }
                for (auto &tm : p.omega[k]) {
                    tw.push_back({tm.z, tm.mask >= 0 ? mp[tm.mask] : nullptr});
                    ky |= galois_of(tm.z) != 1;
                }
                if (kx && sx < 0) { sx = (int)ps.srcs.size(); ps.srcs.push_back(xc + ctw); }
                if (ky && sy < 0) { sy = (int)ps.srcs.size(); ps.srcs.push_back(yc + ctw); }
                ex.add_job(ps, xc, te, sx, nullptr);
                ex.add_job(ps, yc, tw, sy, nullptr);
            }
        }
    }
    std::vector<double *> acc_ptrs(nacc);
    for (int a = 0; a < nacc; ++a) acc_ptrs[a] = acc + (size_t)a * 3 * ctw;
    std::vector<int2> tensor_pairs = req_pairs;
    if (eager) {
        tensor_pairs.resize(npairs);
        for (int q = 0; q < npairs; ++q) tensor_pairs[q] = make_int2(q, 1);
    }
    std::vector<char> extra(tensor_pairs.size() * sizeof(int2) + acc_ptrs.size() * sizeof(void *));
    std::memcpy(extra.data(), tensor_pairs.data(), tensor_pairs.size() * sizeof(int2));
    std::memcpy(extra.data() + tensor_pairs.size() * sizeof(int2), acc_ptrs.data(),
                acc_ptrs.size() * sizeof(void *));

    // --- relinearisation pass: once per product (lazy) or per loop product (eager) ---
    Pass pr;
    std::vector<double *> R(nreq, nullptr);
    std::vector<double *> relin_out;   // the pass's job outputs
    std::vector<char> sums;            // eager: per request (first product, count), then R pointers
    {
        int fi = 0;
        for (int ri = 0; ri < nreq; ++ri)
            R[ri] = info[ri].pe->plan.d > 1 ? rbuf + (size_t)(fi++) * 2 * ctw : reqs[ri].out->d;
        // each job: (c0, c1) of its accumulator with the unrotated term, plus
        // the key switch of c2 (the hoisted source) under the key for s^2
        for (int a = 0; a < nacc; ++a) {
            pr.srcs.push_back(acc_ptrs[a] + 2 * ctw);
            ex.add_job(pr, acc_ptrs[a], {{0, nullptr}}, a, relin_key);
            relin_out.push_back(eager ? ebuf + (size_t)a * 2 * ctw : R[a]);
        }
        if (eager) {
            sums.resize(nreq * sizeof(int2) + nreq * sizeof(void *));
            std::memcpy(sums.data(), req_pairs.data(), nreq * sizeof(int2));
            std::memcpy(sums.data() + nreq * sizeof(int2), R.data(), nreq * sizeof(void *));
        }
    }
    // --- fold pass: C = sum_h Rot(R, h*mo) for the products with d > 1 ---
    Pass pf;
    std::vector<double *> outs;
    for (int ri = 0; ri < nreq; ++ri) {
        const Plan &p = info[ri].pe->plan;
        if (p.d == 1) continue;
        std::vector<std::pair<int, const double *>> terms;
        for (int z : p.fold) terms.push_back({z, nullptr});
        const int src = (int)pf.srcs.size();
        pf.srcs.push_back(R[ri] + ctw);
        ex.add_job(pf, R[ri], terms, src, nullptr);
        outs.push_back(reqs[ri].out->d);
    }
    // the relinearisation pass's table space: its job outputs, then (eager)
    // the per-request sums
    std::vector<char> rextra(relin_out.size() * sizeof(void *) + sums.size());
    std::memcpy(rextra.data(), relin_out.data(), relin_out.size() * sizeof(void *));
    if (!sums.empty()) std::memcpy(rextra.data() + relin_out.size() * sizeof(void *), sums.data(), sums.size());
    std::vector<Exec::Staged> sp;
    const int i_main = nst ? 1 : 0;
    if (nst) sp.push_back({&pst, st_out.data(), st_out.size() * sizeof(void *), Exec::Dev()});
    sp.push_back({&ps, extra.data(), extra.size(), Exec::Dev()});
    sp.push_back({&pr, rextra.data(), rextra.size(), Exec::Dev()});
    if (nfold) sp.push_back({&pf, outs.data(), outs.size() * sizeof(void *), Exec::Dev()});
    ex.stage(sp);

    if (nst) {
        const Exec::Dev &d0 = sp[0].dv;
        if (!ex.launch(d0, nullptr, false, nullptr, Exec::direct_ok(pst) ? (double *const *)d0.extra : nullptr))
            fin_rotsum_launch(T, d0.jobs, d0.terms, d0.E, d0.masks, (double *const *)d0.extra, (int)st_out.size(),
                              st);
    }
    const Exec::Dev &dv = sp[i_main].dv;
    timing.ip_pairs.clear();
    timing.md_pairs.clear();
    Timing lt;
    lt.pooled = true;
    Timing *tm = timing.enabled ? &timing : launch_timing && lt_pairs.size() < LT_MAX ? &lt : nullptr;
    ex.launch(dv, timing.enabled ? ev : nullptr, true, tm);
    if (tm == &lt) {
        lt_pairs.insert(lt_pairs.end(), lt.ip_pairs.begin(), lt.ip_pairs.end());
        lt_md_pairs.insert(lt_md_pairs.end(), lt.md_pairs.begin(), lt.md_pairs.end());
    }
    fin_tensor_launch(T, dv.jobs, dv.terms, dv.E, dv.masks, (const int2 *)dv.extra,
                      (double *const *)(dv.extra + tensor_pairs.size() * sizeof(int2)), nacc, st);
    if (timing.enabled) HGCHK(hipEventRecord(ev[3], st));
    const Exec::Dev &d2 = sp[i_main + 1].dv;
    if (!ex.launch(d2, nullptr, false, nullptr, Exec::direct_ok(pr) ? (double *const *)d2.extra : nullptr))
        fin_rotsum_launch(T, d2.jobs, d2.terms, d2.E, d2.masks, (double *const *)d2.extra, nacc, st);
    if (eager) {
        const char *sm = d2.extra + relin_out.size() * sizeof(void *);
        sum_cts_launch(T, ebuf, (const int2 *)sm, (double *const *)(sm + nreq * sizeof(int2)), nreq, st);
    }
    if (timing.enabled) HGCHK(hipEventRecord(ev[4], st));
    if (nfold) {
        const Exec::Dev &d3 = sp[i_main + 2].dv;
        if (!ex.launch(d3, nullptr, false, nullptr, Exec::direct_ok(pf) ? (double *const *)d3.extra : nullptr))
            fin_rotsum_launch(T, d3.jobs, d3.terms, d3.E, d3.masks, (double *const *)d3.extra, (int)outs.size(), st);
    }
    if (timing.enabled) {
        HGCHK(hipEventRecord(ev[5], st));
        HGCHK(hipEventSynchronize(ev[5]));
        float ms;
        auto el = [&](hipEvent_t a, hipEvent_t b) {
            HGCHK(hipEventElapsedTime(&ms, a, b));
            return (double)ms;
        };
        timing.ms[0] = el(ev[9], ev[0]);
        timing.ms[1] = el(ev[0], ev[1]);
        timing.ms[2] = el(ev[1], ev[2]);
        timing.ms[3] = el(ev[2], ev[3]);
        timing.ms[4] = el(ev[3], ev[4]);
        timing.ms[5] = el(ev[4], ev[5]);
        timing.ms[6] = el(ev[9], ev[5]);
        double ip = 0;
        for (auto &pr : timing.ip_pairs) ip += el(pr.first, pr.second);
        timing.ms[7] = timing.ip_pairs.empty() ? 0.0 : ip / timing.ip_pairs.size();
        timing.ms[8] = (double)timing.ip_pairs.size();
        timing.ip_pairs.clear();
        timing.md_pairs.clear();
        for (auto &x : ev) (void)hipEventDestroy(x);
    }
}

Ct *Ctx::rotate(const Ct &c, int z, hipStream_t st) {
    HGCHK(hipSetDevice(device));
    if (c.comps != 2 || c.ncts != 1) throw Error(-1, "rotate takes one two-component ciphertext");
    need_full_level(c);
    Ct *o = new Ct();
    o->ctx = this;
    ct_alloc(o, st);
    try {
        Exec ex(*this, st);
        Pass ps;
        ps.srcs.push_back(c.d + (size_t)L * N);
        ex.add_job(ps, c.d, {{z, nullptr}}, 0, nullptr);
        double *outp = o->d;
        Exec::Dev dv = ex.run(ps, &outp, sizeof(void *));
        fin_rotsum_launch(T, dv.jobs, dv.terms, dv.E, dv.masks, (double *const *)dv.extra, 1, st);
    } catch (...) {
        delete o;
        throw;
    }
    return o;
}

Ct *Ctx::mul(const Ct &a, const Ct &b, hipStream_t st) {
    HGCHK(hipSetDevice(device));
    if (a.comps != 2 || b.comps != 2 || a.ncts != 1 || b.ncts != 1) throw Error(-1, "mul takes two-component ciphertexts");
    need_full_level(a);
    need_full_level(b);
    const size_t ctw = (size_t)L * N;
    Ct *o = new Ct();
    o->ctx = this;
    ct_alloc(o, st);
    try {
        Exec ex(*this, st);
        double *acc = ex.acc(3 * ctw * sizeof(double));
        Pass ps;
        ex.add_job(ps, a.d, {{0, nullptr}}, -1, nullptr);
        ex.add_job(ps, b.d, {{0, nullptr}}, -1, nullptr);
        struct { int2 rp; double *ap; } ext{make_int2(0, 1), acc};
        static_assert(sizeof(ext) == 16, "layout");
        Exec::Dev dv = ex.run(ps, &ext, sizeof(ext));
        fin_tensor_launch(T, dv.jobs, dv.terms, dv.E, dv.masks, (const int2 *)dv.extra,
                          (double *const *)(dv.extra + 8), 1, st);
        Pass pr;
        pr.srcs.push_back(acc + 2 * ctw);
        ex.add_job(pr, acc, {{0, nullptr}}, 0, relin_key);
        double *outp = o->d;
        Exec::Dev d2 = ex.run(pr, &outp, sizeof(void *));
        fin_rotsum_launch(T, d2.jobs, d2.terms, d2.E, d2.masks, (double *const *)d2.extra, 1, st);
    } catch (...) {
        delete o;
        throw;
    }
    return o;
}

Ct *Ctx::add(const Ct &a, const Ct &b, hipStream_t st) {
    if (a.comps != b.comps || a.ncts != b.ncts) throw Error(-1, "add: mismatched ciphertexts");
    need_full_level(a);
    need_full_level(b);
    Ct *o = new Ct();
    o->ctx = this;
    o->ncts = a.ncts;
    o->comps = a.comps;
    ct_alloc(o, st);
    add_rows(T, o->d, a.d, b.d, a.ncts * a.comps * L, 0, L, st);
    return o;
}

Ct *Ctx::cmul(const Ct &a, const std::vector<uint64_t> &slots, hipStream_t st) {
    need_full_level(a);
    std::vector<uint8_t> key(S);
    // masks are cached by bitmap; general slot values go through a one-off plaintext
    bool binary = true;
    for (int s = 0; s < S; ++s) {
        uint64_t v = s < (int)slots.size() ? slots[s] % t : 0;
        binary &= v <= 1;
        key[s] = (uint8_t)v;
    }
    double *m = nullptr;
    bool own = false;
    if (binary) {
        m = mask_for(key);
    } else {
        double *mu = dev_alloc(N);
        encode_slots(slots, mu, st);
        m = dev_alloc((size_t)nExt * N);
        broadcast_rows(mu, m, N, nExt, st);
        NttArgs na;
        na.out = m; na.in = m; na.rows = nExt; na.per = nExt;
        na.out_stride = na.in_stride = (long long)nExt * N;
        ntt_fwd(T, LOAD_PLAIN, na, st);
        HGCHK(hipStreamSynchronize(st));
        (void)hipFree(mu);
        own = true;
    }
    Ct *o = new Ct();
    o->ctx = this;
    o->ncts = a.ncts;
    o->comps = a.comps;
    ct_alloc(o, st);
    for (int c = 0; c < a.ncts * a.comps; ++c)
        mul_rows(T, o->d + (size_t)c * L * N, a.d + (size_t)c * L * N, m, L, 0, L, st);
    if (own) {
        HGCHK(hipStreamSynchronize(st));
        (void)hipFree(m);
    }
    return o;
}

void Ctx::need_full_level(const Ct &c) const {
    if (c.lv() != L) throw Error(-1, "the ciphertext was modulus-switched: only export and decryption take it");
}

// BGV modulus switching, one prime at a time: from level l to l - 1 the
// input is scaled by k = q_{l-1} mod t (so that the plaintext comes out
// unscaled) and divided by q_{l-1} with the t-corrected rounding of the
// division by P, run by the same kernels with the tables of P = q_{l-1}.
Ct *Ctx::mod_switch(const Ct &c, int drop, hipStream_t st) {
    HGCHK(hipSetDevice(device));
    if (c.comps != 2) throw Error(-1, "modulus switching takes two-component ciphertexts");
    if (drop < 1 || drop >= c.lv()) throw Error(-1, "drop must be at least 1 and leave at least one prime");
    std::unique_ptr<Ct> cur;
    const Ct *in = &c;
    double *scaled = nullptr, *rk = nullptr;
    try {
        scaled = dev_alloc(c.words());
        if (N > 16384) rk = dev_alloc((size_t)c.ncts * 2 * N);
        for (int s = 0; s < drop; ++s) {
            const int l = in->lv();
            const DevTables &M = ms_tabs[l];
            std::unique_ptr<Ct> o(new Ct());
            o->ctx = this;
            o->ncts = in->ncts;
            o->comps = 2;
            o->m = in->m; o->l = in->l; o->n = in->n;
            o->side = in->side;
            o->level = l - 1;
            ct_alloc(o.get(), st);
            const int nslots = in->ncts * 2;
            scale_rows(T, scaled, in->d, nslots * l, l, (double)(qs[l - 1] % t), st);
            if (N <= 16384) {
                moddown_fused(M, o->d, scaled, nslots, st);
            } else {
                NttArgs md;
                md.out = rk;
                md.in = scaled;
                md.rows = nslots;
                md.per = 1;
                md.prime_base = l - 1;
                md.out_stride = (long long)N;
                md.in_stride = (long long)l * N;
                md.in_offset = (long long)(l - 1) * N;
                ntt_inv(M, STORE_MDR, md, st);
                NttArgs dl;
                dl.out = o->d;
                dl.in = rk;
                dl.aux = scaled;
                dl.rows = nslots * (l - 1);
                dl.in_stride = (long long)N;
                ntt_fwd(M, LOAD_DELTA, dl, st);
            }
            cur = std::move(o);   // the steps run in stream order on the shared scratch
            in = cur.get();
        }
        HGCHK(hipStreamSynchronize(st));
    } catch (...) {
        (void)hipStreamSynchronize(st);
        if (scaled) (void)hipFree(scaled);
        if (rk) (void)hipFree(rk);
        throw;
    }
    (void)hipFree(scaled);
    if (rk) (void)hipFree(rk);
    return cur.release();
}

}  // namespace hg
