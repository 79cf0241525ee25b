// Continuous-batching request loop (see server.h).
#include "server.h"

#include <algorithm>
#include <cstring>

namespace hg {

Footprint request_footprint_parts(const Ctx &C, const Plan &p) {
    const uint64_t w = 8, N = C.N, L = C.L, nExt = C.nExt, beta = C.beta, alpha = C.alpha;
    const uint64_t ct = 2 * L * N * w;
    // key-switched jobs of the transform pass: transforms with a rotated term
    // (one division by P each), or every rotated term in the paper's order
    uint64_t nks = 0;
    auto count = [&](const std::vector<Term> &tms) {
        uint64_t rot = 0;
        for (auto &t : tms) rot += ((t.z % C.S) + C.S) % C.S != 0;
        if (!rot) return (uint64_t)0;
        const bool lone = tms.size() == 1 && tms[0].mask < 0;
        return C.ks_order == 1 && !lone ? rot : (uint64_t)1;
    };
    for (int k = 0; k < p.K; ++k) nks += count(p.eps[k]) + count(p.omega[k]);
    nks *= (uint64_t)p.nb;
    const uint64_t nsrc = 2 * (uint64_t)p.nb;
    const uint64_t operands = 2 * (uint64_t)p.nb * ct;
    const uint64_t result = ct;
    uint64_t acc = 3 * L * N * w + (p.d > 1 ? ct : 0) + (p.method == 3 ? 2 * ct : 0);
    uint64_t scratch = nsrc * (L + beta * nExt) * N * w + nks * 2 * (nExt + alpha + L) * N * w;
    if (p.method == 3) {
        uint64_t nst = count(p.sigma) + count(p.tau);
        scratch = std::max(scratch, 2 * (L + beta * nExt) * N * w + nst * 2 * (nExt + alpha + L) * N * w);
    }
    if (C.relin == 1) {
        // eager relinearisation: a tensor and a relinearised ciphertext per
        // loop product, and a relinearisation pass with one source and one
        // key switch per loop product
        const uint64_t pairs = (uint64_t)p.nb * p.K;
        acc += pairs * 5 * L * N * w;
        scratch = std::max(scratch, pairs * (L + beta * nExt) * N * w + pairs * 2 * (nExt + alpha + L) * N * w);
    }
    Footprint f;
    // a lane's device buffer: the operands as read (canonical words), the
    // operands in evaluation form, and the result
    f.buffers = 2 * operands + result;
    // the executor's workspaces (exactly sized on server lanes), plus their
    // rounding to whole MiB and the descriptor tables
    f.workspace = acc + scratch + (3ull << 20);
    return f;
}

uint64_t request_footprint(const Ctx &C, const Plan &p) {
    const Footprint f = request_footprint_parts(C, p);
    return f.buffers + f.workspace;
}

Server::Server(Ctx &c, const ServerConfig &cf) : C(c), cfg(cf), lanes(cf.lanes) {
    if (cfg.max_batch < 1 || cfg.lanes < 1 || cfg.lanes > 8) throw Error(-1, "server: bad configuration");
    HGCHK(hipSetDevice(C.device));
    for (auto &ln : lanes) {
        HGCHK(hipStreamCreateWithFlags(&ln.st, hipStreamNonBlocking));
        HGCHK(hipEventCreateWithFlags(&ln.done, hipEventDisableTiming));
        // workspaces sized exactly (the admission model counts them so)
        C.arena(ln.st).exact = true;
    }
    origin = std::chrono::steady_clock::now();
    th = std::thread([this] { loop(); });
    ++C.servers;
}

Server::~Server() {
    {
        std::lock_guard<std::mutex> g(mu);
        stop = true;
        paused = false;   // destroy finishes every submitted request
    }
    cv_sub.notify_all();
    if (th.joinable()) th.join();
    --C.servers;
    (void)hipSetDevice(C.device);
    for (auto &ln : lanes) {
        if (ln.st) (void)hipStreamSynchronize(ln.st);
        if (ln.done) (void)hipEventDestroy(ln.done);
        // the executor's scratch arena of this stream goes with the stream
        auto it = C.arenas.find(ln.st);
        if (it != C.arenas.end()) {
            it->second.release();
            C.arenas.erase(it);
        }
        auto ax = C.aux.find(ln.st);
        if (ax != C.aux.end()) {
            if (ax->second.side) (void)hipStreamSynchronize(ax->second.side);
            for (auto &ring : ax->second.ev)
                for (hipEvent_t e : ring) (void)hipEventDestroy(e);
            if (ax->second.side) (void)hipStreamDestroy(ax->second.side);
            C.aux.erase(ax);
        }
        if (ln.st) (void)hipStreamDestroy(ln.st);
    }
    for (auto &kv : reqs)
        if (kv.second->pin) (void)hipHostFree(kv.second->pin);
    for (auto &kv : pool) (void)hipHostFree(kv.second);
}

uint64_t *Server::pin_get(size_t words, size_t &cap) {
    {
        std::lock_guard<std::mutex> g(pool_mu);
        auto it = pool.lower_bound(words);
        if (it != pool.end() && it->first <= 2 * words) {
            uint64_t *p = it->second;
            cap = it->first;
            pool.erase(it);
            return p;
        }
    }
    void *p = nullptr;
    HGCHK(hipHostMalloc(&p, words * sizeof(uint64_t), hipHostMallocDefault));
    cap = words;
    return (uint64_t *)p;
}

void Server::pin_put(uint64_t *p, size_t cap) {
    std::lock_guard<std::mutex> g(pool_mu);
    if (pool.size() < 256) {
        pool.emplace(cap, p);
        return;
    }
    (void)hipHostFree(p);
}

double Server::now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - origin).count();
}

uint64_t Server::submit(const uint64_t *a, size_t na, const uint64_t *b, size_t nbw, int m, int l, int n) {
    if (!a || !b) throw Error(-1, "null operand");
    if (m <= 0 || l <= 0 || n <= 0) throw Error(-1, "dimensions must be positive");
    // plans and keys are made by hg_keygen before serving; look up only
    auto it = C.plans.find(std::make_tuple(m, l, n));
    if (it == C.plans.end()) throw Error(-3, "shape has no plan and keys (list it in hg_keygen)");
    const PlanEntry *pe = it->second.get();
    if (!pe->keys_found.load(std::memory_order_relaxed)) {
        for (int z : pe->plan.rotations(C.S))
            if (!C.rot_key(C.galois_of(z))) throw Error(-3, "missing rotation key for z = " + std::to_string(z));
        pe->keys_found.store(true, std::memory_order_relaxed);
    }
    const size_t ctw = (size_t)2 * C.L * C.N;
    const size_t want = (size_t)pe->plan.nb * ctw;
    if (na != want || nbw != want) throw Error(-1, "operand word count differs from the shape's packing");
    for (int side = 0; side < 2; ++side) {
        const uint64_t *w = side ? b : a;
        for (size_t r = 0; r < want / C.N; ++r) {
            const uint64_t q = C.qs[r % C.L];
            const uint64_t *row = w + r * C.N;
            for (int i = 0; i < C.N; ++i)
                if (row[i] >= q) throw Error(-1, "residue out of range");
        }
    }
    auto rq = std::make_unique<Req>();
    rq->m = m;
    rq->l = l;
    rq->n = n;
    rq->pe = pe;
    rq->na = na;
    rq->nb = nbw;
    rq->nc = ctw;
    rq->pin = pin_get(na + nbw + ctw, rq->pin_cap);
    std::memcpy(rq->pin, a, na * sizeof(uint64_t));
    std::memcpy(rq->pin + na, b, nbw * sizeof(uint64_t));
    rq->fp = request_footprint_parts(C, pe->plan);
    uint64_t id;
    {
        std::lock_guard<std::mutex> g(mu);
        id = next_id++;
        rq->id = id;
        rq->t_submit = now();
        pending.push_back(rq.get());
        reqs[id] = std::move(rq);
    }
    cv_sub.notify_one();
    return id;
}

void Server::wait(uint64_t id, uint64_t *c, size_t nc, double *times) {
    std::unique_ptr<Req> rq;
    {
        std::unique_lock<std::mutex> g(mu);
        auto it = reqs.find(id);
        if (it == reqs.end()) throw Error(-1, "unknown ticket");
        Req *r = it->second.get();
        cv_done.wait(g, [&] { return r->status == 2 || r->status < 0; });
        rq = std::move(it->second);
        reqs.erase(it);
    }
    struct Release {   // the pinned buffer goes back to the pool on every path
        Server *s;
        Req *r;
        ~Release() { s->pin_put(r->pin, r->pin_cap); }
    } release{this, rq.get()};
    if (rq->status < 0) throw Error(rq->status, rq->err);
    if (times) {
        times[0] = rq->t_submit;
        times[1] = rq->t_start;
        times[2] = rq->t_done;
    }
    if (c) {
        if (nc < rq->nc) throw Error(-1, "result buffer too small");
        std::memcpy(c, rq->pin + rq->na + rq->nb, rq->nc * sizeof(uint64_t));
    }
}

void Server::pause(bool p) {
    {
        std::lock_guard<std::mutex> g(mu);
        paused = p;
    }
    cv_sub.notify_all();
}

void Server::stats(double *o) {
    std::lock_guard<std::mutex> g(mu);
    o[0] = (double)n_done;
    o[1] = (double)n_batches;
    o[2] = n_batches ? sum_batch / n_batches : 0.0;
    o[3] = (double)max_inflight;
    o[4] = (double)max_overlap;
    o[5] = (double)pending.size();
    o[6] = (double)inflight;
    o[7] = now();
}

void Server::launch(Lane &ln, std::vector<Req *> &batch) {
    const hipStream_t st = ln.st;
    const size_t N = C.N, L = C.L;
    const size_t ctw = 2 * L * N;
    size_t in_words = 0;
    for (Req *r : batch) in_words += r->na + r->nb;
    const size_t out_words = batch.size() * ctw;
    // device buffer: operands (in_words doubles), results (out_words
    // doubles), canonical staging (in_words words; in_words >= 2 out_words)
    char *dbuf = nullptr;
    HGCHK(hipMallocAsync((void **)&dbuf, (2 * in_words + out_words) * 8, st));
    try {
        launch_group(ln, batch, dbuf, in_words, out_words);
    } catch (...) {
        (void)hipFreeAsync(dbuf, st);
        throw;
    }
    HGCHK(hipFreeAsync(dbuf, st));
    HGCHK(hipEventRecord(ln.done, st));
}

void Server::launch_group(Lane &ln, std::vector<Req *> &batch, char *dbuf, size_t in_words, size_t out_words) {
    const hipStream_t st = ln.st;
    const size_t N = C.N, L = C.L;
    const size_t ctw = 2 * L * N;
    double *ops = (double *)dbuf;
    double *outs = ops + in_words;
    uint64_t *stage = (uint64_t *)(outs + out_words);
    size_t o = 0;
    for (Req *r : batch) {   // straight from each request's pinned buffer
        HGCHK(hipMemcpyAsync(stage + o, r->pin, (r->na + r->nb) * 8, hipMemcpyHostToDevice, st));
        o += r->na + r->nb;
    }
    u64_to_dbl(stage, ops, in_words, st);
    NttArgs a;
    a.out = ops;
    a.in = ops;
    a.rows = (int)(in_words / N);
    a.per = (int)L;
    a.out_stride = a.in_stride = (long long)(L * N);
    ntt_fwd(C.T, LOAD_PLAIN, a, st);

    ln.cts.clear();
    std::vector<Ctx::Request> rq;
    o = 0;
    for (size_t i = 0; i < batch.size(); ++i) {
        Req *r = batch[i];
        const Plan &p = r->pe->plan;
        auto mk = [&](double *d, int side, int ncts) {
            auto c = std::make_unique<Ct>();
            c->ctx = &C;
            c->owns = false;
            c->ncts = ncts;
            c->comps = 2;
            c->m = r->m;
            c->l = r->l;
            c->n = r->n;
            c->side = side;
            c->d = d;
            ln.cts.push_back(std::move(c));
            return ln.cts.back().get();
        };
        Ct *A = mk(ops + o, side_of_role(p, 0), p.nb);
        o += r->na;
        Ct *B = mk(ops + o, side_of_role(p, 1), p.nb);
        o += r->nb;
        Ct *Cc = mk(outs + i * ctw, 2, 1);
        rq.push_back({A, B, r->m, r->l, r->n, Cc});
    }
    C.hegmm_batch_window(rq, st);
    // results to canonical words (the operand region is free by now)
    NttArgs e;
    e.out = ops;
    e.in = outs;
    e.rows = (int)(out_words / N);
    e.per = (int)L;
    e.out_stride = e.in_stride = (long long)(L * N);
    ntt_inv(C.T, STORE_CANON, e, st);
    dbl_to_u64(ops, stage, out_words, st);
    for (size_t i = 0; i < batch.size(); ++i)
        HGCHK(hipMemcpyAsync(batch[i]->pin + batch[i]->na + batch[i]->nb, stage + i * ctw, ctw * 8,
                             hipMemcpyDeviceToHost, st));
}

void Server::finish(Lane &ln, int code, const std::string &msg) {
    const double t = now();
    {
        std::lock_guard<std::mutex> g(mu);
        for (size_t i = 0; i < ln.batch.size(); ++i) {
            Req *r = ln.batch[i];
            r->t_done = t;
            if (code == 0) {
                r->status = 2;
                ++n_done;
            } else {
                r->status = code;
                r->err = msg;
            }
        }
        inflight -= ln.buffers;
    }
    ln.buffers = 0;
    ln.batch.clear();
    ln.cts.clear();
    ln.busy = false;
    cv_done.notify_all();
}

void Server::loop() {
    (void)hipSetDevice(C.device);
    for (;;) {
        bool progressed = false;
        // 1. completed groups
        for (auto &ln : lanes) {
            if (!ln.busy) continue;
            const hipError_t e = hipEventQuery(ln.done);
            if (e == hipSuccess) {
                finish(ln, 0, "");
                progressed = true;
            } else if (e != hipErrorNotReady) {
                finish(ln, -5, std::string("device error: ") + hipGetErrorString(e));
                progressed = true;
            }
        }
        // 2. admit pending requests in arrival order onto free lanes
        for (auto &ln : lanes) {
            if (ln.busy) continue;
            std::vector<Req *> batch;
            uint64_t bufs = 0, work = 0, held = ln.held;
            {
                std::lock_guard<std::mutex> g(mu);
                bool busy_lanes = false;
                for (auto &o : lanes) busy_lanes |= o.busy;
                while (!paused && !pending.empty() && (int)batch.size() < cfg.max_batch) {
                    Req *r = pending.front();
                    // the lane keeps the larger of its workspace and this group's
                    const uint64_t h = std::max(ln.held, work + r->fp.workspace);
                    const uint64_t after = inflight - ln.held + h + bufs + r->fp.buffers;
                    const bool fits = cfg.budget == 0 || after <= cfg.budget ||
                                      (!busy_lanes && batch.empty());   // a lone request always runs
                    if (!fits) break;
                    pending.pop_front();
                    bufs += r->fp.buffers;
                    work += r->fp.workspace;
                    held = h;
                    batch.push_back(r);
                }
                if (batch.empty()) break;
                inflight = inflight - ln.held + held + bufs;
                ln.held = held;
                max_inflight = std::max(max_inflight, inflight);
                const double t = now();
                for (Req *r : batch) {
                    r->status = 1;
                    r->t_start = t;
                }
                ++n_batches;
                sum_batch += (double)batch.size();
                uint64_t busy = 1;
                for (auto &o : lanes) busy += o.busy;
                max_overlap = std::max(max_overlap, busy);
            }
            ln.batch = batch;
            ln.buffers = bufs;
            ln.busy = true;
            try {
                launch(ln, ln.batch);
            } catch (Error &e) {
                (void)hipStreamSynchronize(ln.st);
                finish(ln, e.code, e.what());
            } catch (std::exception &e) {
                (void)hipStreamSynchronize(ln.st);
                finish(ln, -1, e.what());
            }
            progressed = true;
        }
        // 3. leave when stopped and drained; otherwise wait for work
        std::unique_lock<std::mutex> g(mu);
        bool any_busy = false;
        for (auto &ln : lanes) any_busy |= ln.busy;
        if (stop && pending.empty() && !any_busy) break;
        if (progressed) continue;
        if (any_busy)
            cv_sub.wait_for(g, std::chrono::microseconds(20));
        else
            cv_sub.wait(g, [&] { return stop || (!paused && !pending.empty()); });
    }
}

}  // namespace hg
