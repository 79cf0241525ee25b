// Continuous-batching request loop for HE matrix products.
//
// Clients submit serialised operand ciphertexts (the canonical words a
// client sends to the cloud, Algorithm 2's hand-over); a server thread admits
// pending requests in arrival order while their modelled device footprint
// fits the budget, launches each admitted group with the batched executor on
// one of several streams ("lanes"), so that groups overlap on the device, and
// returns each result as canonical words.  Requests that arrive while others
// run are admitted as soon as a lane and memory are free.  Every result is
// the bit pattern that the product gives alone.
#pragma once
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "context.h"

namespace hg {

// Modelled device bytes a product of this plan holds while it runs:
// `buffers`, its operands (as received and in evaluation form) and result,
// released when its group finishes; `workspace`, its accumulator and its
// share of the pass scratch (hoisted digits, inner-product outputs,
// division-by-P buffers, tables), which a lane keeps for its later groups.
struct Footprint {
    uint64_t buffers = 0, workspace = 0;
};
Footprint request_footprint_parts(const Ctx &C, const Plan &p);
uint64_t request_footprint(const Ctx &C, const Plan &p);   // buffers + workspace

struct ServerConfig {
    int max_batch = 64;       // products per launch group
    int lanes = 2;            // launch groups in flight, one stream each
    uint64_t budget = 0;      // modelled bytes of in-flight requests (0: unlimited)
};

struct Server {
    struct Req {
        uint64_t id = 0;
        int m = 0, l = 0, n = 0;
        const PlanEntry *pe = nullptr;
        // pinned host buffer: operand words a then b (copied in by submit),
        // then the result's words (copied out of the device by the lane)
        uint64_t *pin = nullptr;
        size_t pin_cap = 0, na = 0, nb = 0, nc = 0;
        Footprint fp;
        double t_submit = 0, t_start = 0, t_done = 0;
        int status = 0;                  // 0 queued, 1 running, 2 done, < 0 error code
        std::string err;
    };
    struct Lane {
        hipStream_t st = nullptr;
        hipEvent_t done = nullptr;
        bool busy = false;
        std::vector<Req *> batch;
        std::vector<std::unique_ptr<Ct>> cts;   // non-owning views of the lane's device buffer
        uint64_t buffers = 0;   // modelled bytes of the in-flight group's buffer
        uint64_t held = 0;      // modelled workspace the lane keeps (largest group so far)
    };

    Ctx &C;
    ServerConfig cfg;
    std::vector<Lane> lanes;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv_sub, cv_done;
    std::deque<Req *> pending;
    std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
    uint64_t next_id = 1;
    bool stop = false;
    bool paused = false;     // admission held (requests queue up)
    // modelled device bytes now: every lane's kept workspace plus the
    // buffers of the groups in flight (guarded by mu)
    uint64_t inflight = 0;
    std::chrono::steady_clock::time_point origin;
    // pool of pinned request buffers, reused by size (guarded by pool_mu)
    std::mutex pool_mu;
    std::multimap<size_t, uint64_t *> pool;
    uint64_t *pin_get(size_t words, size_t &cap);
    void pin_put(uint64_t *p, size_t cap);
    // statistics (guarded by mu)
    uint64_t n_done = 0, n_batches = 0, max_inflight = 0, max_overlap = 0;
    double sum_batch = 0;

    Server(Ctx &c, const ServerConfig &cf);
    ~Server();

    uint64_t submit(const uint64_t *a, size_t na, const uint64_t *b, size_t nb, int m, int l, int n);
    // blocks until the request is done; fills c (result words) and times
    // (submit, start, done; seconds since the server started)
    void wait(uint64_t id, uint64_t *c, size_t nc, double *times);
    void stats(double *out8);
    // hold (true) or resume (false) admission; queued requests wait meanwhile
    void pause(bool p);

  private:
    double now() const;
    void loop();
    void launch(Lane &ln, std::vector<Req *> &batch);
    void launch_group(Lane &ln, std::vector<Req *> &batch, char *dbuf, size_t in_words, size_t out_words);
    void finish(Lane &ln, int code, const std::string &msg);
};



}  // namespace hg
