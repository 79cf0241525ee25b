// extern "C" entry points declared in include/hegmm.h.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>

#include "../../include/hegmm.h"
#include "context.h"
#include "server.h"

struct hg_ctx {
    hg::Ctx *c;
};
struct hg_ct {
    hg::Ct *c;
};
struct hg_server {
    hg::Server *s;
};
struct hg_graph {
    hg::Graph *g;
};

namespace {

thread_local std::string g_err;

template <class F>
hg_status guard(F &&f) {
    try {
        f();
        return HG_OK;
    } catch (hg::Error &e) {
        g_err = e.what();
        return e.code;
    } catch (std::bad_alloc &) {
        g_err = "host allocation failed";
        return HG_ENOMEM;
    } catch (std::exception &e) {
        g_err = e.what();
        return HG_EINVAL;
    }
}

void need(bool cond, const char *msg) {
    if (!cond) throw hg::Error(HG_EINVAL, msg);
}

hg_ct *wrap(hg::Ct *c) {
    hg_ct *h = new hg_ct;
    h->c = c;
    return h;
}

hipStream_t as_stream(void *s) { return (hipStream_t)s; }

// While a request server runs, its thread owns the context: every other call
// that reads or changes the context's state is refused.
void unowned(const hg::Ctx &X) {
    if (X.servers > 0)
        throw hg::Error(HG_ESTATE, "a server owns this context: only hg_server_* and hg_request_footprint may be "
                                   "called until hg_server_destroy");
}

}  // namespace

// ---------------------------------------------------------------------------
// Workspace of hg_hegmm_noalloc: one fixed device array per GPU, reserved
// when the library's code object is loaded on that GPU and held until the
// process ends.  In host code `scratch` names a host-side stand-in, not
// device memory: its device address on the current GPU comes from
// hipGetSymbolAddress, looked up once per device when a context is created
// there, and only that address is handed to kernels.
// ---------------------------------------------------------------------------
#define HG_NOALLOC_TABLE_BYTES (1ull << 20)
static __device__ __align__(256) unsigned char scratch[HG_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::map<int, char *> g_scratch_ptr;   // device -> its copy of `scratch`

// The device address of `scratch` on `dev` (which must be current).
char *scratch_on(int dev) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) return it->second;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        throw hg::Error(HG_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = (char *)ptr;
    return (char *)ptr;
}

// Set up a context's fixed arena over the device's scratch, with its own
// pinned staging for descriptor tables (made here, at creation, so that the
// allocation-free entry point never allocates).
void noalloc_setup(hg::Ctx &X) {
    hg::Arena &a = X.noalloc_arena;
    a.fixed_base = scratch_on(X.device);
    a.fixed_bytes = HG_NOALLOC_SCRATCH_BYTES;
    HGCHK(hipEventCreateWithFlags(&a.staged, hipEventDisableTiming));
    HGCHK(hipHostMalloc(&a.pinned, HG_NOALLOC_TABLE_BYTES, hipHostMallocDefault));
    HGCHK(hipHostGetDevicePointer(&a.pinned_dev, a.pinned, 0));
    a.pinned_cap = HG_NOALLOC_TABLE_BYTES;
}

}  // namespace

extern "C" {

const char *hg_last_error(void) { return g_err.c_str(); }

hg_status hg_set_allocator(hg_ctx *ctx, hg_alloc_fn alloc, hg_release_fn release, void *user) {
    return guard([&] {
        need(ctx, "null argument");
        unowned(*ctx->c);
        need((alloc == nullptr) == (release == nullptr), "alloc and release must be given together");
        hg::Ctx &X = *ctx->c;
        X.ct_alloc_fn = alloc;
        X.ct_release_fn = release;
        X.ct_alloc_user = alloc ? user : nullptr;
    });
}

hg_status hg_ctx_create(const hg_params *p, int dev, hg_ctx **out) {
    return guard([&] {
        need(p && out, "null argument");
        *out = nullptr;
        need(p->min_blocks <= 4096, "min_blocks out of range");
        need(p->method <= 3, "method must be 0, 1, 2 or 3");
        need(p->min_blocks <= 1 || p->method == 0 || p->method == 2, "forced blocking needs HEGMM-En (method 2)");
        need(p->relin <= 1, "relin must be 0 (lazy) or 1 (eager)");
        need(p->ks_order <= 1, "ks_order must be 0 (one division by P per transform) or 1 (per rotation)");
        need(p->prime_bits == 0 || (p->prime_bits >= 32 && p->prime_bits <= 50), "prime_bits must be 0 or in [32, 50]");
        need(p->sigma == 0.0 || p->sigma == 3.2, "sigma must be 0 or 3.2 (the sampler's table is fixed for 3.2)");
        hg::Ctx *c = new hg::Ctx(p->N, p->t, p->L, p->alpha, dev, p->method == 0 ? 2 : (int)p->method,
                                 p->prime_bits ? (int)p->prime_bits : 50);
        c->min_blocks = p->min_blocks > 1 ? (int)p->min_blocks : 1;
        c->relin = (int)p->relin;
        c->ks_order = (int)p->ks_order;
        try {
            noalloc_setup(*c);
        } catch (...) {
            delete c;
            throw;
        }
        hg_ctx *h = new hg_ctx;
        h->c = c;
        *out = h;
    });
}

void hg_ctx_destroy(hg_ctx *ctx) {
    if (!ctx) return;
    delete ctx->c;
    delete ctx;
}

hg_status hg_keygen(hg_ctx *ctx, uint64_t seed, const int32_t *shapes, size_t nshapes) {
    return guard([&] {
        need(ctx && (shapes || nshapes == 0), "null argument");
        unowned(*ctx->c);
        hg::Ctx &C = *ctx->c;
        HGCHK(hipSetDevice(C.device));
        std::vector<int> gal;
        auto add = [&](int m, int l, int n) {
            const hg::PlanEntry &pe = C.plan_for(m, l, n);
            for (int z : pe.plan.rotations(C.S)) gal.push_back(C.galois_of(z));
        };
        for (size_t i = 0; i < nshapes; ++i) {
            const int m = shapes[3 * i], l = shapes[3 * i + 1], n = shapes[3 * i + 2];
            if (const hg::Ctx::Partition *pt = C.partition_for(m, l, n)) {
                for (int mi : pt->rows)
                    for (int nj : pt->cols) add(mi, l, nj);
            } else {
                add(m, l, n);
            }
        }
        C.keygen(seed, gal);
    });
}

hg_status hg_keygen_rotations(hg_ctx *ctx, const int32_t *z, size_t count) {
    return guard([&] {
        need(ctx && (z || count == 0), "null argument");
        unowned(*ctx->c);
        hg::Ctx &C = *ctx->c;
        if (!C.has_secret) throw hg::Error(HG_ESTATE, "keygen with a seed first");
        HGCHK(hipSetDevice(C.device));
        std::vector<int> gal;
        for (size_t i = 0; i < count; ++i) gal.push_back(C.galois_of(z[i]));
        C.keygen(C.seed, gal);
    });
}

hg_status hg_drop_secret(hg_ctx *ctx) {
    return guard([&] {
        need(ctx, "null context");
        unowned(*ctx->c);
        ctx->c->drop_secret();
    });
}

hg_status hg_encrypt(hg_ctx *ctx, int role, const int64_t *X, int m, int l, int n, uint64_t nonce, hg_ct **out) {
    return guard([&] {
        need(ctx && X && out, "null argument");
        unowned(*ctx->c);
        *out = nullptr;
        need(m > 0 && l > 0 && n > 0, "dimensions must be positive");
        hg::Ctx &C = *ctx->c;
        HGCHK(hipSetDevice(C.device));
        if (const hg::Ctx::Partition *pt = C.partition_for(m, l, n))
            *out = wrap(C.encrypt_blocked(role, X, m, l, n, nonce, *pt));
        else
            *out = wrap(C.encrypt_matrix(role, X, m, l, n, nonce));
    });
}

hg_status hg_set_partition(hg_ctx *ctx, int m, int l, int n, const int32_t *rows, int nrows, const int32_t *cols,
                           int ncols) {
    return guard([&] {
        need(ctx && rows && cols && nrows > 0 && ncols > 0, "null argument or empty partition");
        unowned(*ctx->c);
        ctx->c->set_partition(m, l, n, std::vector<int>(rows, rows + nrows), std::vector<int>(cols, cols + ncols));
    });
}

hg_status hg_get_partition(hg_ctx *ctx, int m, int l, int n, int32_t *out, size_t cap, size_t *count) {
    return guard([&] {
        need(ctx && count, "null argument");
        unowned(*ctx->c);
        const hg::Ctx::Partition *pt = ctx->c->partition_for(m, l, n);
        std::vector<int32_t> v{pt ? (int32_t)pt->rows.size() : 1, pt ? (int32_t)pt->cols.size() : 1};
        if (pt) {
            v.insert(v.end(), pt->rows.begin(), pt->rows.end());
            v.insert(v.end(), pt->cols.begin(), pt->cols.end());
        } else {
            v.push_back(m);
            v.push_back(n);
        }
        *count = v.size();
        if (!out) return;
        need(cap >= v.size(), "buffer too small");
        std::copy(v.begin(), v.end(), out);
    });
}

hg_status hg_hegmm_batch(hg_ctx *ctx, size_t cnt, const hg_ct *const *A, const hg_ct *const *B, const int32_t *mln,
                         hg_ct **C, void *stream) {
    std::vector<hg::Ct *> made;
    hg_status st = guard([&] {
        need(ctx && A && B && mln && C, "null argument");
        unowned(*ctx->c);
        hg::Ctx &X = *ctx->c;
        HGCHK(hipSetDevice(X.device));
        std::vector<hg::Ctx::Request> reqs;
        std::vector<std::unique_ptr<hg::Ct>> views;   // block operands and results of output-blocked products
        for (size_t i = 0; i < cnt; ++i) {
            need(A[i] && B[i], "null operand");
            need(A[i]->c->ctx == &X && B[i]->c->ctx == &X, "operand from another context");
            const int m = mln[3 * i], l = mln[3 * i + 1], n = mln[3 * i + 2];
            need(m > 0 && l > 0 && n > 0, "dimensions must be positive");
            const hg::Ctx::Partition *pt = X.partition_for(m, l, n);
            hg::Ct *o = new hg::Ct();
            o->ctx = &X;
            o->ncts = pt ? pt->blocks() : 1;
            o->comps = 2;
            o->m = m; o->l = l; o->n = n;
            o->side = pt ? 12 : 2;
            made.push_back(o);
            X.ct_alloc(o, as_stream(stream));
            if (!pt) {
                reqs.push_back({A[i]->c, B[i]->c, m, l, n, o});
                continue;
            }
            // one product per output block, on views into the blocked operands
            const hg::Ct &a = *A[i]->c, &b = *B[i]->c;
            need(a.side == 10 && b.side == 11 && a.m == m && a.l == l && a.n == n && b.m == m && b.l == l && b.n == n,
                 "operands must be hg_encrypt outputs of this output-blocked shape for roles 0 (A) and 1 (B)");
            int first = 0, k = 0;
            for (int mi : pt->rows)
                for (int nj : pt->cols) {
                    const hg::Plan &p = X.plan_for(mi, l, nj).plan;
                    auto view = [&](const hg::Ct &src, int side, int ncts, int at) {
                        auto v = std::make_unique<hg::Ct>();
                        v->ctx = &X;
                        v->owns = false;
                        v->ncts = ncts;
                        v->comps = 2;
                        v->m = mi; v->l = l; v->n = nj;
                        v->side = side;
                        v->d = src.ct(at);
                        views.push_back(std::move(v));
                        return views.back().get();
                    };
                    need(first + p.nb <= a.ncts && first + p.nb <= b.ncts, "blocked operand too short");
                    hg::Ct *va = view(a, hg::side_of_role(p, 0), p.nb, first);
                    hg::Ct *vb = view(b, hg::side_of_role(p, 1), p.nb, first);
                    hg::Ct *vc = view(*o, 2, 1, k);
                    reqs.push_back({va, vb, mi, l, nj, vc});
                    first += p.nb;
                    ++k;
                }
            need(first == a.ncts && first == b.ncts, "blocked operand of another partition");
        }
        X.hegmm_batch(reqs, as_stream(stream));
    });
    if (st != HG_OK) {
        for (auto *o : made) delete o;
        return st;
    }
    for (size_t i = 0; i < cnt; ++i) C[i] = wrap(made[i]);
    return HG_OK;
}

hg_status hg_hegmm_noalloc(hg_ctx *ctx, const hg_ct *ctA, const hg_ct *ctB, int m, int l, int n, hg_ct *ctC,
                           void *stream) {
    return guard([&] {
        need(ctx && ctA && ctB && ctC, "null argument");
        unowned(*ctx->c);
        hg::Ctx &X = *ctx->c;
        need(ctA->c->ctx == &X && ctB->c->ctx == &X && ctC->c->ctx == &X, "handle from another context");
        need(m > 0 && l > 0 && n > 0, "dimensions must be positive");
        need(ctC != ctA && ctC != ctB && ctC->c->d != ctA->c->d && ctC->c->d != ctB->c->d,
             "the result handle must not be an operand");
        hg::Ct &R = *ctC->c;
        need(R.ncts == 1 && R.comps == 2 && R.level == 0 && R.d,
             "the result handle must hold one two-component ciphertext at the full level");
        need(!X.partitions.count(std::make_tuple(m, l, n)), "output-blocked products are not supported here");
        // a plan not made yet would allocate its masks: hg_keygen makes them
        if (!X.plans.count(std::make_tuple(m, l, n)))
            throw hg::Error(HG_ESTATE, "shape not prepared: list it in hg_keygen before hg_hegmm_noalloc");
        HGCHK(hipSetDevice(X.device));
        std::vector<hg::Ctx::Request> reqs{{ctA->c, ctB->c, m, l, n, &R}};
        // neither timing mode (events, waits) nor the pipelined passes (a
        // second stream) run here; the batch is one launch window
        const bool timing = X.timing.enabled, lt = X.launch_timing;
        const int pipeline = X.pipeline;
        X.timing.enabled = false;
        X.launch_timing = false;
        X.pipeline = 1;
        X.fixed_arena = &X.noalloc_arena;
        try {
            X.hegmm_batch_window(reqs, as_stream(stream));
        } catch (...) {
            X.fixed_arena = nullptr;
            X.timing.enabled = timing;
            X.launch_timing = lt;
            X.pipeline = pipeline;
            throw;
        }
        X.fixed_arena = nullptr;
        X.timing.enabled = timing;
        X.launch_timing = lt;
        X.pipeline = pipeline;
        R.m = m;
        R.l = l;
        R.n = n;
        R.side = 2;
    });
}

hg_status hg_graph_create(hg_ctx *ctx, size_t cnt, const hg_ct *const *A, const hg_ct *const *B, const int32_t *mln,
                          hg_ct **C, hg_graph **out) {
    std::vector<hg::Ct *> made;
    hg::Graph *gr = nullptr;
    hg_status st = guard([&] {
        need(ctx && A && B && mln && C && out, "null argument");
        unowned(*ctx->c);
        need(cnt > 0, "empty batch");
        *out = nullptr;
        hg::Ctx &X = *ctx->c;
        HGCHK(hipSetDevice(X.device));
        std::vector<hg::Ctx::Request> reqs;
        for (size_t i = 0; i < cnt; ++i) {
            need(A[i] && B[i], "null operand");
            need(A[i]->c->ctx == &X && B[i]->c->ctx == &X, "operand from another context");
            need(mln[3 * i] > 0 && mln[3 * i + 1] > 0 && mln[3 * i + 2] > 0, "dimensions must be positive");
            hg::Ct *o = new hg::Ct();
            o->ctx = &X;
            o->ncts = 1;
            o->comps = 2;
            o->m = mln[3 * i]; o->l = mln[3 * i + 1]; o->n = mln[3 * i + 2];
            o->side = 2;
            made.push_back(o);
            X.ct_alloc(o, nullptr);
            reqs.push_back({A[i]->c, B[i]->c, mln[3 * i], mln[3 * i + 1], mln[3 * i + 2], o});
        }
        gr = new hg::Graph(X, reqs);
    });
    if (st != HG_OK) {
        for (auto *o : made) delete o;
        return st;
    }
    for (size_t i = 0; i < cnt; ++i) C[i] = wrap(made[i]);
    *out = new hg_graph{gr};
    return HG_OK;
}

hg_status hg_graph_launch(hg_graph *g, void *stream) {
    return guard([&] {
        need(g, "null graph");
        unowned(*g->g->C);
        g->g->launch(as_stream(stream));
    });
}

void hg_graph_destroy(hg_graph *g) {
    if (!g) return;
    delete g->g;
    delete g;
}

hg_status hg_ct_load(hg_ctx *ctx, hg_ct *ct, const uint64_t *buf, size_t nwords, void *stream) {
    return guard([&] {
        need(ctx && ct && buf, "null argument");
        unowned(*ctx->c);
        hg::Ctx &X = *ctx->c;
        need(ct->c->ctx == &X, "handle from another context");
        HGCHK(hipSetDevice(X.device));
        X.load_ct(*ct->c, buf, nwords, as_stream(stream));
    });
}

hg_status hg_hegmm(hg_ctx *ctx, const hg_ct *ctA, const hg_ct *ctB, int m, int l, int n, hg_ct **ctC, void *stream) {
    if (ctC) *ctC = nullptr;
    int32_t mln[3] = {m, l, n};
    return hg_hegmm_batch(ctx, 1, &ctA, &ctB, mln, ctC, stream);
}

hg_status hg_decrypt(hg_ctx *ctx, const hg_ct *ct, int m, int l, int n, uint64_t *C) {
    return guard([&] {
        need(ctx && ct && C, "null argument");
        unowned(*ctx->c);
        hg::Ctx &X = *ctx->c;
        const hg::Ct &R = *ct->c;
        need(m > 0 && l > 0 && n > 0, "dimensions must be positive");
        const hg::Ctx::Partition *pt = X.partition_for(m, l, n);
        const int ncts = pt ? pt->blocks() : 1;
        const bool result = R.side == (pt ? 12 : 2) && R.m == m && R.l == l && R.n == n;
        // hg_ct_import of a result's words
        const bool imported = R.side == -1 && R.ncts == ncts && R.comps == 2;
        need(result || imported, "not a result of this shape");
        HGCHK(hipSetDevice(X.device));
        HGCHK(hipDeviceSynchronize());
        if (!pt) {
            const hg::PlanEntry &pe = X.plan_for(m, l, n);
            std::vector<uint64_t> slots = X.decrypt_slot_values(*ct->c, 0);
            for (int i = 0; i < m; ++i)
                for (int j = 0; j < n; ++j) C[(size_t)i * n + j] = slots[hg::result_slot(pe.plan, i, j)];
            return;
        }
        // output blocks: block k = (i, j) holds C's rows r0.., columns c0..
        int k = 0, r0 = 0;
        for (int mi : pt->rows) {
            int c0 = 0;
            for (int nj : pt->cols) {
                const hg::PlanEntry &pe = X.plan_for(mi, l, nj);
                std::vector<uint64_t> slots = X.decrypt_slot_values(*ct->c, k);
                for (int i = 0; i < mi; ++i)
                    for (int j = 0; j < nj; ++j)
                        C[(size_t)(r0 + i) * n + c0 + j] = slots[hg::result_slot(pe.plan, i, j)];
                ++k;
                c0 += nj;
            }
            r0 += mi;
        }
    });
}

hg_status hg_ct_export(hg_ctx *ctx, const hg_ct *ct, uint64_t *buf, size_t nwords, size_t *needed) {
    return guard([&] {
        need(ctx && ct, "null argument");
        unowned(*ctx->c);
        const size_t w = ct->c->words();
        if (needed) *needed = w;
        if (!buf) return;
        need(nwords >= w, "buffer too small");
        HGCHK(hipSetDevice(ctx->c->device));
        HGCHK(hipDeviceSynchronize());
        ctx->c->export_ct(*ct->c, buf, nullptr);
    });
}

hg_status hg_ct_import(hg_ctx *ctx, const uint64_t *buf, size_t nwords, int ncts, int comps, hg_ct **out) {
    return guard([&] {
        need(ctx && buf && out, "null argument");
        unowned(*ctx->c);
        *out = nullptr;
        need(ncts > 0 && (comps == 2 || comps == 3), "bad ciphertext count or component count");
        hg::Ctx &X = *ctx->c;
        need(nwords == (size_t)ncts * comps * X.L * X.N, "word count does not match");
        HGCHK(hipSetDevice(X.device));
        *out = wrap(X.import_ct(buf, ncts, comps, nullptr));
    });
}

void hg_ct_free(hg_ct *ct) {
    if (!ct) return;
    delete ct->c;
    delete ct;
}

hg_status hg_encrypt_slots(hg_ctx *ctx, const int64_t *slots, uint64_t nonce, hg_ct **out) {
    return guard([&] {
        need(ctx && slots && out, "null argument");
        unowned(*ctx->c);
        *out = nullptr;
        hg::Ctx &X = *ctx->c;
        HGCHK(hipSetDevice(X.device));
        std::vector<uint64_t> v(X.S);
        for (int s = 0; s < X.S; ++s) {
            int64_t r = slots[s] % (int64_t)X.t;
            v[s] = (uint64_t)(r < 0 ? r + (int64_t)X.t : r);
        }
        *out = wrap(X.encrypt_slots(v, 2, 0, nonce));
    });
}

hg_status hg_decrypt_slots(hg_ctx *ctx, const hg_ct *ct, uint64_t *slots) {
    return guard([&] {
        need(ctx && ct && slots, "null argument");
        unowned(*ctx->c);
        hg::Ctx &X = *ctx->c;
        HGCHK(hipSetDevice(X.device));
        HGCHK(hipDeviceSynchronize());
        std::vector<uint64_t> v = X.decrypt_slot_values(*ct->c, 0);
        std::memcpy(slots, v.data(), v.size() * sizeof(uint64_t));
    });
}

hg_status hg_rotate(hg_ctx *ctx, const hg_ct *ct, int z, hg_ct **out, void *stream) {
    return guard([&] {
        need(ctx && ct && out, "null argument");
        unowned(*ctx->c);
        *out = nullptr;
        *out = wrap(ctx->c->rotate(*ct->c, z, as_stream(stream)));
    });
}

hg_status hg_mul(hg_ctx *ctx, const hg_ct *a, const hg_ct *b, hg_ct **out, void *stream) {
    return guard([&] {
        need(ctx && a && b && out, "null argument");
        unowned(*ctx->c);
        *out = nullptr;
        *out = wrap(ctx->c->mul(*a->c, *b->c, as_stream(stream)));
    });
}

hg_status hg_add(hg_ctx *ctx, const hg_ct *a, const hg_ct *b, hg_ct **out, void *stream) {
    return guard([&] {
        need(ctx && a && b && out, "null argument");
        unowned(*ctx->c);
        *out = nullptr;
        *out = wrap(ctx->c->add(*a->c, *b->c, as_stream(stream)));
    });
}

hg_status hg_mod_switch(hg_ctx *ctx, const hg_ct *ct, int drop, hg_ct **out, void *stream) {
    return guard([&] {
        need(ctx && ct && out, "null argument");
        unowned(*ctx->c);
        *out = nullptr;
        *out = wrap(ctx->c->mod_switch(*ct->c, drop, as_stream(stream)));
    });
}

hg_status hg_cmul(hg_ctx *ctx, const hg_ct *a, const int64_t *slots, hg_ct **out, void *stream) {
    return guard([&] {
        need(ctx && a && slots && out, "null argument");
        unowned(*ctx->c);
        *out = nullptr;
        hg::Ctx &X = *ctx->c;
        std::vector<uint64_t> v(X.S);
        for (int s = 0; s < X.S; ++s) {
            int64_t r = slots[s] % (int64_t)X.t;
            v[s] = (uint64_t)(r < 0 ? r + (int64_t)X.t : r);
        }
        *out = wrap(X.cmul(*a->c, v, as_stream(stream)));
    });
}

hg_status hg_plan_info(hg_ctx *ctx, int m, int l, int n, int64_t *out) {
    return guard([&] {
        need(ctx && out, "null argument");
        unowned(*ctx->c);
        hg::Ctx &X = *ctx->c;
        hg::Plan p;
        try {
            p = hg::make_plan(m, l, n, X.S, X.method, X.min_blocks);
        } catch (std::invalid_argument &e) {
            throw hg::Error(HG_EINVAL, e.what());
        } catch (std::range_error &e) {
            throw hg::Error(HG_ENOFIT, e.what());
        }
        out[0] = p.transposed;
        out[1] = p.nb;
        out[2] = p.lb;
        out[3] = p.d;
        out[4] = p.M;
        out[5] = p.K;
        out[6] = p.W;
        out[7] = (int64_t)p.rotations(X.S).size();
        out[8] = (int64_t)p.masks.size();
        out[9] = p.key_switched_terms(X.S);
    });
}

hg_status hg_primes(hg_ctx *ctx, uint64_t *out) {
    return guard([&] {
        need(ctx && out, "null argument");
        for (size_t i = 0; i < ctx->c->qs.size(); ++i) out[i] = ctx->c->qs[i];
    });
}

hg_status hg_tune(hg_ctx *ctx, const char *name, int64_t value) {
    return guard([&] {
        need(ctx && name, "null argument");
        need(value >= 0 && value < (1LL << 30), "value out of range");
        hg::Ctx &X = *ctx->c;
        if (X.servers > 0) throw hg::Error(HG_ESTATE, "a server owns this context; tune it before hg_server_create");
        const std::string n(name);
        // transform knobs live in the context's tables (and those of its
        // modulus-switching divisions), so contexts do not share them
        auto set_tables = [&](int hg::DevTables::*field, int v) {
            X.T.*field = v;
            for (auto &M : X.ms_tabs) M.*field = v;
        };
        if (n == "fuse_rows") X.fuse_rows = (int)value;
        else if (n == "ip_chunk") X.ip_chunk = (int)value;
        else if (n == "ip_order") X.ip_order = (int)value;
        else if (n == "split_rows") set_tables(&hg::DevTables::split_rows, (int)value);
        else if (n == "half_rows") set_tables(&hg::DevTables::half_rows, (int)value);
        else if (n == "xcd_rows") {
            need(value == 0 || value == 1, "xcd_rows must be 0 or 1");
            set_tables(&hg::DevTables::xcd_rows, (int)value);
        }
        else if (n == "ntt_radix") {
            need(value == 0 || value == 8 || value == 16, "ntt_radix must be 0, 8 or 16");
            set_tables(&hg::DevTables::row_rk, hg::ntt_radix_rk((int)value));
        }
        else if (n == "batch_window") X.batch_window = (int)value;
        else if (n == "pipeline") {
            need(value >= 1 && value <= 16, "pipeline must be in [1, 16]");
            X.pipeline = (int)value;
        }
        else throw hg::Error(HG_EINVAL, "unknown tuning knob " + n);
    });
}

hg_status hg_set_timing(hg_ctx *ctx, int enable) {
    return guard([&] {
        need(ctx, "null context");
        unowned(*ctx->c);
        need(enable >= 0 && enable <= 2, "timing mode must be 0, 1 or 2");
        ctx->c->timing.enabled = enable == 1;
        ctx->c->launch_timing = enable == 2;
    });
}

hg_status hg_launch_timing(hg_ctx *ctx, double *out4) {
    return guard([&] {
        need(ctx && out4, "null argument");
        unowned(*ctx->c);
        hg::Ctx &X = *ctx->c;
        HGCHK(hipSetDevice(X.device));
        auto read = [&](std::vector<std::pair<hipEvent_t, hipEvent_t>> &v, double *o) {
            double sum = 0;
            for (auto &pr : v) {
                HGCHK(hipEventSynchronize(pr.second));
                float ms = 0;
                HGCHK(hipEventElapsedTime(&ms, pr.first, pr.second));
                sum += ms;
            }
            o[0] = v.empty() ? 0.0 : sum / v.size();
            o[1] = (double)v.size();
            for (auto &pr : v) {
                X.lt_free.push_back(pr.first);
                X.lt_free.push_back(pr.second);
            }
            v.clear();
        };
        read(X.lt_pairs, out4);
        read(X.lt_md_pairs, out4 + 2);
    });
}

hg_status hg_last_timing(hg_ctx *ctx, double *out9) {
    return guard([&] {
        need(ctx && out9, "null argument");
        unowned(*ctx->c);
        for (int i = 0; i < 9; ++i) out9[i] = ctx->c->timing.ms[i];
    });
}

hg_status hg_request_footprint(hg_ctx *ctx, int m, int l, int n, uint64_t *bytes) {
    return guard([&] {
        need(ctx && bytes, "null argument");
        hg::Ctx &X = *ctx->c;
        hg::Plan p;
        try {
            p = hg::make_plan(m, l, n, X.S, X.method, X.min_blocks);
        } catch (std::invalid_argument &e) {
            throw hg::Error(HG_EINVAL, e.what());
        } catch (std::range_error &e) {
            throw hg::Error(HG_ENOFIT, e.what());
        }
        *bytes = hg::request_footprint(X, p);
    });
}

hg_status hg_server_create(hg_ctx *ctx, const hg_server_config *cfg, hg_server **out) {
    return guard([&] {
        need(ctx && cfg && out, "null argument");
        unowned(*ctx->c);
        *out = nullptr;
        hg::ServerConfig sc;
        sc.max_batch = cfg->max_batch;
        sc.lanes = cfg->lanes;
        sc.budget = cfg->hbm_budget;
        hg::Server *s = new hg::Server(*ctx->c, sc);
        *out = new hg_server{s};
    });
}

hg_status hg_server_submit(hg_server *srv, const uint64_t *a_words, size_t a_nwords, const uint64_t *b_words,
                           size_t b_nwords, int m, int l, int n, uint64_t *ticket) {
    return guard([&] {
        need(srv && ticket, "null argument");
        *ticket = srv->s->submit(a_words, a_nwords, b_words, b_nwords, m, l, n);
    });
}

hg_status hg_server_wait(hg_server *srv, uint64_t ticket, uint64_t *c_words, size_t c_nwords, double *times3) {
    return guard([&] {
        need(srv, "null server");
        srv->s->wait(ticket, c_words, c_nwords, times3);
    });
}

hg_status hg_server_pause(hg_server *srv, int paused) {
    return guard([&] {
        need(srv, "null server");
        need(paused == 0 || paused == 1, "paused must be 0 or 1");
        srv->s->pause(paused == 1);
    });
}

hg_status hg_server_stats(hg_server *srv, double *out8) {
    return guard([&] {
        need(srv && out8, "null argument");
        srv->s->stats(out8);
    });
}

void hg_server_destroy(hg_server *srv) {
    if (!srv) return;
    delete srv->s;
    delete srv;
}

}  // extern "C"
