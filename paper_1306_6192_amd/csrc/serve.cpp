// Serving runtime: continuous batching of arriving products.
//
// A scheduler thread owns the device side.  Clients submit problems (copied
// into a FIFO with a ticket); the scheduler loops over
//   retire  -- poll the completion event of every running batch, stamp its
//              requests done and give back their footprint and slots;
//   admit   -- move requests from the FIFO head into the admitted list while
//              the sum of in-flight footprints stays within the HBM budget
//              and the in-flight count within max_inflight;
//   launch  -- on every idle stream, take up to max_batch admitted requests
//              of one mode (the oldest request's) and run them as one grouped
//              persistent launch, then record an event.
// Batches on different streams run concurrently on the device, and requests
// that arrive while others run are admitted as soon as footprint and slots
// free up.  A problem gets the same tile configuration (a function of its
// shape) whatever batch it lands in, so its result does not depend on the mix.
//
// Executors: 0 = GPU (grouped launches), 1 = host fake (no HIP call; batches
// finish after a short simulated time, every Nth batch may be made to fail),
// 2 = GPU plain launches, one per request, in FIFO order on one stream (the
// unbatched baseline).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "grouped.hpp"

namespace mg {

enum ReqState { Q_QUEUED = 0, Q_ADMITTED = 1, Q_RUNNING = 2, Q_DONE = 3 };

struct Request {
    uint64_t ticket;
    gemm_problem_t p;
    uint64_t footprint;
    uint64_t t_arrival = 0, t_admit = 0, t_launch = 0, t_done = 0;
    int32_t status = GEMM_PENDING;
    int32_t batch_size = 0;
    int state = Q_QUEUED;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    DevBuf descs;
    void *host = nullptr;
    size_t host_bytes = 0;
    DevBuf ws;                           // split-K workspace (plain executor)
    std::vector<Request *> running;      // empty = idle
    uint64_t fake_done_at = 0;
    bool fake_fail = false;
};

// Device bytes a request holds while in flight: its operands and output,
// plus, under the plain-launch executor, the workspace its plain launch uses
// (split-K partial slabs, split-BF16x3 operand copies).  Grouped launches use
// no workspace.
static uint64_t footprint_of(const gemm_problem_t &p, int executor) {
    const uint64_t es = elem_size(p.mode);
    uint64_t fp = (uint64_t)p.m * p.k * es + (uint64_t)p.k * p.n * es + (uint64_t)p.m * p.n * 4;
    if (executor == 2 && p.m > 0 && p.n > 0 && p.k > 0) {
        int c = 0, sp = 1;
        tuner_choose(p.mode, p.m, p.n, p.k, &c, &sp);
        fp += (uint64_t)plain_ws_bytes(p, c, sp);
    }
    return fp;
}

struct Server {
    gemm_serve_config_t cfg;
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work;   // wakes the scheduler
    std::condition_variable cv_done;   // wakes drain()
    std::deque<Request *> queue;
    std::deque<Request *> admitted;
    std::unordered_map<uint64_t, Request *> by_ticket;
    std::vector<Slot> slots;
    uint64_t next_ticket = 1;
    uint64_t inflight_bytes = 0, peak_bytes = 0;
    int inflight = 0;
    uint64_t submitted = 0, completed = 0, failed = 0, batches = 0;
    bool stop = false;
    int sticky = GEMM_OK;              // a HIP failure puts the server in a failed state
    std::thread thread;

    int init();
    void loop();
    void retire_locked(uint64_t now);
    void admit_locked(uint64_t now);
    void launch_locked(uint64_t now);
    int launch_batch(Slot &s, std::vector<Request *> &b);
    void finish_locked(Request *r, int status, uint64_t now);
    void fail_all_locked(int status, uint64_t now);
    bool busy_locked() const;
};

bool Server::busy_locked() const {
    if (!queue.empty() || !admitted.empty()) return true;
    for (const Slot &s : slots)
        if (!s.running.empty()) return true;
    return false;
}

int Server::init() {
    if (cfg.executor != 1) {
        MG_HIP(hipGetDevice(&device));
    }
    slots.resize(cfg.executor == 2 ? 1 : cfg.num_streams);
    if (cfg.executor != 1) {
        for (Slot &s : slots) {
            MG_HIP(hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
            MG_HIP(hipEventCreateWithFlags(&s.done, hipEventDisableTiming));
        }
    }
    thread = std::thread([this] { loop(); });
    return GEMM_OK;
}

void Server::finish_locked(Request *r, int status, uint64_t now) {
    r->status = status;
    r->t_done = now;
    r->state = Q_DONE;
    inflight_bytes -= r->footprint;
    inflight -= 1;
    if (status == GEMM_OK) ++completed;
    else ++failed;
}

void Server::fail_all_locked(int status, uint64_t now) {
    for (Slot &s : slots) {
        for (Request *r : s.running) finish_locked(r, status, now);
        s.running.clear();
    }
    for (Request *r : admitted) finish_locked(r, status, now);
    admitted.clear();
    for (Request *r : queue) {
        r->status = status;
        r->t_done = now;
        r->state = Q_DONE;
        ++failed;
    }
    queue.clear();
}

void Server::retire_locked(uint64_t now) {
    for (Slot &s : slots) {
        if (s.running.empty()) continue;
        int status = GEMM_OK;
        if (cfg.executor == 1) {
            if (now < s.fake_done_at) continue;
            if (s.fake_fail) status = GEMM_EINTERNAL;
        } else {
            const hipError_t e = hipEventQuery(s.done);
            if (e == hipErrorNotReady) continue;
            if (e != hipSuccess) {
                status = GEMM_EHIP;
                sticky = GEMM_EHIP;
            }
        }
        for (Request *r : s.running) finish_locked(r, status, now);
        s.running.clear();
    }
    if (sticky != GEMM_OK) fail_all_locked(sticky, now);
}

void Server::admit_locked(uint64_t now) {
    while (!queue.empty()) {
        Request *r = queue.front();
        if (inflight >= cfg.max_inflight) break;
        if (inflight_bytes + r->footprint > cfg.hbm_budget_bytes) break;   // FIFO: no overtaking
        queue.pop_front();
        r->state = Q_ADMITTED;
        r->t_admit = now;
        inflight += 1;
        inflight_bytes += r->footprint;
        peak_bytes = std::max(peak_bytes, inflight_bytes);
        admitted.push_back(r);
    }
}

int Server::launch_batch(Slot &s, std::vector<Request *> &b) {
    if (cfg.executor == 1) {
        // simulated device time: 1 us per request plus 1 us per GFLOP
        double gflop = 0;
        for (Request *r : b) gflop += 2e-9 * (double)r->p.m * r->p.n * r->p.k;
        s.fake_done_at = now_ns() + 1000ull * b.size() + (uint64_t)(gflop * 1000.0);
        s.fake_fail = cfg.fake_fail_every > 0 && (batches % (uint64_t)cfg.fake_fail_every) ==
                                                     (uint64_t)(cfg.fake_fail_every - 1);
        return GEMM_OK;
    }
    if (cfg.executor == 2) {
        for (Request *r : b) {
            int c = 0, sp = 1;
            tuner_choose(r->p.mode, r->p.m, r->p.n, r->p.k, &c, &sp);
            const int64_t need = plain_ws_bytes(r->p, c, sp);
            if (need > 0) {
                int rc = s.ws.ensure((size_t)need, s.stream);
                if (rc != GEMM_OK) return rc;
            }
            int rc = enqueue_plain(r->p, c, sp, s.ws.ptr, s.stream);
            if (rc != GEMM_OK) return rc;
        }
        MG_HIP(hipEventRecord(s.done, s.stream));
        return GEMM_OK;
    }
    if (b.size() == 1) {
        // A batch of one runs as a plain launch of one of the grouped kernel's
        // tile configurations (no split: the same bits as in a batch),
        // without the descriptor upload; alone, the tile that spreads the
        // product over the most CUs may finish first.
        const gemm_problem_t &p = b[0]->p;
        const GroupedKernel *gk = grouped_kernel(p.mode);
        if (!gk) return fail(GEMM_EUNSUPPORTED, "mode %d has no grouped kernel", p.mode);
        const int cfg = gk->alone_idx[grouped_choose_alone(p.mode, p.m, p.n, p.k)];
        int rc = enqueue_plain(p, cfg, 1, nullptr, s.stream);
        if (rc != GEMM_OK) return rc;
        MG_HIP(hipEventRecord(s.done, s.stream));
        return GEMM_OK;
    }
    std::vector<gemm_problem_t> ps;
    ps.reserve(b.size());
    for (Request *r : b) ps.push_back(r->p);
    GroupPlan plan;
    int rc = build_group_plan(ps.data(), (int)ps.size(), plan);
    if (rc != GEMM_OK) return rc;
    if (plan.total_tiles > 0) {
        const size_t bytes = plan_image_bytes(plan);
        rc = s.descs.ensure(std::max<size_t>(bytes, 4096), s.stream);
        if (rc != GEMM_OK) return rc;
        if (s.host_bytes < bytes) {
            if (s.host) MG_HIP(hipHostFree(s.host));
            s.host = nullptr;
            s.host_bytes = 0;
            MG_HIP(hipHostMalloc(&s.host, std::max<size_t>(bytes, 65536), hipHostMallocDefault));
            s.host_bytes = std::max<size_t>(bytes, 65536);
        }
        // the slot is idle: its previous upload has completed
        plan_image_write(plan, s.host);
        MG_HIP(hipMemcpyAsync(s.descs.ptr, s.host, bytes, hipMemcpyHostToDevice, s.stream));
        rc = enqueue_group(plan, s.descs.ptr, s.stream);
        if (rc != GEMM_OK) return rc;
    }
    MG_HIP(hipEventRecord(s.done, s.stream));
    return GEMM_OK;
}

void Server::launch_locked(uint64_t now) {
    for (Slot &s : slots) {
        if (admitted.empty()) return;
        if (!s.running.empty()) continue;
        const int mode = admitted.front()->p.mode;
        const int cap = std::max(1, cfg.max_batch);
        std::vector<Request *> b;
        for (auto it = admitted.begin(); it != admitted.end() && (int)b.size() < cap;) {
            if ((*it)->p.mode == mode) {
                b.push_back(*it);
                it = admitted.erase(it);
            } else {
                ++it;
            }
        }
        for (Request *r : b) {
            r->state = Q_RUNNING;
            r->t_launch = now;
            r->batch_size = (int32_t)b.size();
        }
        const int rc = launch_batch(s, b);
        ++batches;
        if (rc != GEMM_OK) {
            const uint64_t t = now_ns();
            for (Request *r : b) finish_locked(r, rc, t);
            if (rc == GEMM_EHIP) {
                sticky = GEMM_EHIP;
                fail_all_locked(sticky, t);
                return;
            }
            continue;
        }
        s.running = std::move(b);
    }
}

void Server::loop() {
    if (cfg.executor != 1) (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
        const uint64_t now = now_ns();
        retire_locked(now);
        admit_locked(now);
        launch_locked(now);
        cv_done.notify_all();
        bool running = false;
        for (Slot &s : slots) running |= !s.running.empty();
        if (stop && !busy_locked()) break;
        if (running) {
            // device work in flight: poll its events.  The scheduler thread
            // spins (yielding) rather than sleeping: a timed sleep on Linux
            // lasts tens of microseconds, more than many requests take.
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        } else if (queue.empty() && admitted.empty()) {
            cv_work.wait(lk, [this] { return stop || !queue.empty(); });
        }
    }
    cv_done.notify_all();
}

}  // namespace mg

using namespace mg;

extern "C" {

int gemm_serve_footprint(const gemm_problem_t *p, uint64_t *bytes_out) {
    clear_error();
    if (!bytes_out) return fail(GEMM_EINVAL, "bytes_out is NULL");
    int rc = validate(p);
    if (rc != GEMM_OK) return rc;
    *bytes_out = footprint_of(*p, 0);
    return GEMM_OK;
}

int gemm_serve_create(const gemm_serve_config_t *cfg, void **server_out) {
    clear_error();
    if (!cfg || !server_out) return fail(GEMM_EINVAL, "NULL argument");
    *server_out = nullptr;
    if (cfg->max_inflight < 1 || cfg->num_streams < 1 || cfg->max_batch < 1 || cfg->queue_capacity < 1 ||
        cfg->hbm_budget_bytes == 0)
        return fail(GEMM_EINVAL, "serve config: every limit must be positive");
    if (cfg->num_streams > 16) return fail(GEMM_EINVAL, "serve config: at most 16 streams");
    if (cfg->executor < 0 || cfg->executor > 2) return fail(GEMM_EINVAL, "unknown executor %d", cfg->executor);
    if (cfg->fake_fail_every < 0) return fail(GEMM_EINVAL, "fake_fail_every must be >= 0");
    Server *s = new Server();
    s->cfg = *cfg;
    int rc = s->init();
    if (rc != GEMM_OK) {
        for (Slot &sl : s->slots) {
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
        }
        delete s;
        return rc;
    }
    *server_out = s;
    return GEMM_OK;
}

int gemm_serve_submit(void *server, const gemm_problem_t *p, uint64_t t_arrival_ns, uint64_t *ticket_out) {
    clear_error();
    if (!server || !ticket_out) return fail(GEMM_EINVAL, "NULL argument");
    Server *s = static_cast<Server *>(server);
    int rc = validate(p);
    if (rc != GEMM_OK) return rc;
    const uint64_t fp = footprint_of(*p, s->cfg.executor);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->sticky != GEMM_OK) return fail(s->sticky, "server is in a failed state");
    if (s->stop) return fail(GEMM_EINVAL, "server is shutting down");
    if (fp > s->cfg.hbm_budget_bytes)
        return fail(GEMM_ENOMEM, "footprint %llu exceeds the budget %llu", (unsigned long long)fp,
                    (unsigned long long)s->cfg.hbm_budget_bytes);
    if ((int)s->queue.size() >= s->cfg.queue_capacity) return fail(GEMM_EBUSY, "queue full");
    Request *r = new Request();
    r->ticket = s->next_ticket++;
    r->p = *p;
    r->footprint = fp;
    r->t_arrival = t_arrival_ns ? t_arrival_ns : now_ns();
    s->queue.push_back(r);
    s->by_ticket[r->ticket] = r;
    ++s->submitted;
    *ticket_out = r->ticket;
    s->cv_work.notify_one();
    return GEMM_OK;
}

int gemm_serve_poll(void *server, uint64_t ticket, gemm_serve_result_t *out) {
    clear_error();
    if (!server || !out) return fail(GEMM_EINVAL, "NULL argument");
    Server *s = static_cast<Server *>(server);
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->by_ticket.find(ticket);
    if (it == s->by_ticket.end()) return fail(GEMM_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Request *r = it->second;
    if (r->state != Q_DONE) return GEMM_PENDING;
    out->status = r->status;
    out->batch_size = r->batch_size;
    out->t_arrival_ns = r->t_arrival;
    out->t_admit_ns = r->t_admit;
    out->t_launch_ns = r->t_launch;
    out->t_done_ns = r->t_done;
    const int st = r->status;
    s->by_ticket.erase(it);
    delete r;
    if (st != GEMM_OK) return fail(st, "request failed");
    return GEMM_OK;
}

int gemm_serve_drain(void *server) {
    clear_error();
    if (!server) return fail(GEMM_EINVAL, "NULL server");
    Server *s = static_cast<Server *>(server);
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_work.notify_one();
    s->cv_done.wait(lk, [s] { return !s->busy_locked(); });
    return s->sticky;
}

int gemm_serve_stats(void *server, gemm_serve_stats_t *out) {
    clear_error();
    if (!server || !out) return fail(GEMM_EINVAL, "NULL argument");
    Server *s = static_cast<Server *>(server);
    std::lock_guard<std::mutex> lk(s->mu);
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->failed = s->failed;
    out->batches = s->batches;
    out->inflight_bytes = s->inflight_bytes;
    out->peak_inflight_bytes = s->peak_bytes;
    out->queued = (int32_t)s->queue.size();
    out->inflight = s->inflight;
    return GEMM_OK;
}

int gemm_serve_destroy(void *server) {
    clear_error();
    if (!server) return fail(GEMM_EINVAL, "NULL server");
    Server *s = static_cast<Server *>(server);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_one();
    }
    s->thread.join();
    for (Slot &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        sl.descs.release();
        sl.ws.release();
        if (sl.host) (void)hipHostFree(sl.host);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    for (auto &kv : s->by_ticket) delete kv.second;
    delete s;
    return GEMM_OK;
}

// Open-loop load generator: submit ps[i] at t0 + offsets_ns[i] (t0 = the
// call time), stamping the scheduled time as its arrival, so queueing delay
// counts in the latency even when the submitting thread falls behind.  A
// full queue is retried until accepted.  Blocks until every request is
// submitted (not completed).
int gemm_serve_replay(void *server, const gemm_problem_t *ps, const uint64_t *offsets_ns, int32_t count,
                      uint64_t *tickets_out) {
    clear_error();
    if (!server || (count > 0 && (!ps || !offsets_ns || !tickets_out))) return fail(GEMM_EINVAL, "NULL argument");
    const uint64_t t0 = now_ns();
    for (int32_t i = 0; i < count; ++i) {
        const uint64_t due = t0 + offsets_ns[i];
        while (now_ns() < due) {
        }
        while (true) {
            const int rc = gemm_serve_submit(server, &ps[i], due, &tickets_out[i]);
            if (rc == GEMM_OK) break;
            if (rc != GEMM_EBUSY) return rc;
            std::this_thread::sleep_for(std::chrono::microseconds(5));
        }
    }
    return GEMM_OK;
}

}  // extern "C"
