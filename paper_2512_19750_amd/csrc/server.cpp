// server.cpp -- the serving loop behind gace_server_*.
//
// Tables stay resident in device memory (owned by the caller); requests arrive
// from any thread.  A worker thread keeps up to `max_inflight` batches on the
// device, each on its own stream and context (own workspace slot): whenever a
// slot is free and requests are waiting, it admits queued requests in arrival
// order while their estimated workspace fits the slot, compiles them into one
// batch and launches it, even while the other slots' batches are still running
// (continuous batching).  A request finishes as soon as its own scan or join
// does: the kernels publish each finished scan's and join's results into the
// slot's pinned result buffer and raise a host flag, which the worker polls;
// the batch's done event finishes whatever has not published (scans with no
// items, or every request after a device error).  Each request's outputs and
// status are written once and its waiter woken.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "runtime.h"
#include "../../include/gace_zone.h"

namespace {

struct OwnedRequest {
    gace_request r;
    std::vector<gace_column> cols;
    std::vector<gace_term> terms;
    std::vector<uint32_t> pred_off;
    uint64_t ticket = 0;
    uint64_t ws_est = 0;
};

struct ServeSlot {
    gace_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    bool busy = false;
    gace::CompiledBatch cb;
    std::vector<std::unique_ptr<OwnedRequest>> reqs;
    std::vector<gace_request> arr;
    std::vector<gace_status> per;
    std::vector<char> fin;                                  // request finished before its batch
    std::vector<std::pair<uint32_t, gace_status>> ready;    // requests finished by the last poll
    uint64_t ws = 0;
};

struct TicketState {
    bool done = false;
    gace_status st = GACE_OK;
    uint64_t submit_ns = 0, done_ns = 0;   // CLOCK_MONOTONIC
};

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// device bytes a join needs: its partitioned key buffer (8 bytes per sampled
// key, bounded by the expected kept blocks plus 12 standard deviations) and
// its per-item partition tables
uint64_t join_bytes(const gace_request& r) {
    uint64_t U = 0;
    const gace_keys* s[2] = {&r.R, &r.S};
    for (int i = 0; i < 2; ++i) {
        const uint64_t B = s[i]->spec.block_rows ? s[i]->spec.block_rows : 1;
        const uint64_t nb = (s[i]->n + B - 1) / B;
        const uint64_t thr = gace::rate_threshold(s[i]->spec.rate);
        double p = thr >= gace::kThrAll ? 1.0 : (double)thr / 4294967296.0;
        double kept = (double)nb * p + 12.0 * std::sqrt((double)nb * p * (1.0 - p)) + 16.0;
        uint64_t k = kept >= (double)nb ? nb : (uint64_t)kept;
        U += std::min<uint64_t>(s[i]->n, k * B);
    }
    // partitioned keys and the first-pass buffer (8 + 8 bytes per key), the
    // per-item partition counts (at most U / 8 bytes) and chunk tables of
    // partitions split by hot keys (about 8 bytes per key for Zipf-skewed keys)
    return 24 * U + U / 8 + (1ull << 20);
}

}  // namespace

struct gace_server {
    gace_server_cfg cfg{};
    int device = 0;
    std::vector<ServeSlot> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::unique_ptr<OwnedRequest>> queue;
    std::unordered_map<uint64_t, TicketState> tickets;
    uint64_t next_ticket = 1;
    uint64_t slot_budget = 0;
    bool stop = false;
    std::thread worker;
    gace_server_stats stats{};
    std::vector<const gace_zonemap*> zonemaps;   // attached zone maps, copied to a slot at each launch

    void run();
    bool try_complete(ServeSlot& s, std::unique_lock<std::mutex>& lk);
    bool try_launch(ServeSlot& s, std::unique_lock<std::mutex>& lk);
};

// A running batch: requests whose scan or join has published its results
// (per-request completion) are finished at once; the rest when the batch's
// done event fires.
bool gace_server::try_complete(ServeSlot& s, std::unique_lock<std::mutex>& lk) {
    if (!s.busy) return false;
    hipError_t q = hipEventQuery(s.ctx->ev_done);
    if (q == hipErrorNotReady) {
        s.ready.clear();
        gace::collect_published(s.ctx, s.cb, s.arr.data(), s.fin, s.ready);
        if (s.ready.empty()) return false;
        const uint64_t t_done = now_ns();
        for (const auto& rs : s.ready) {
            TicketState& t = tickets[s.reqs[rs.first]->ticket];
            t.done = true;
            t.st = rs.second;
            t.done_ns = t_done;
        }
        stats.completed += s.ready.size();
        stats.completed_early += s.ready.size();
        stats.inflight -= s.ready.size();
        cv_done.notify_all();
        return true;
    }
    lk.unlock();
    if (q == hipSuccess) {
        (void)gace::finish_compiled(s.ctx, s.cb, s.arr.data(), s.per.data(), &s.fin);
    } else {
        for (auto& p : s.per) p = GACE_EDEVICE;
    }
    lk.lock();
    const uint64_t t_done = now_ns();
    size_t n_late = 0;
    for (size_t i = 0; i < s.reqs.size(); ++i) {
        if (s.fin[i]) continue;
        OwnedRequest& o = *s.reqs[i];
        TicketState& t = tickets[o.ticket];
        t.done = true;
        t.st = s.per[i];
        t.done_ns = t_done;
        ++n_late;
    }
    stats.completed += n_late;
    stats.inflight -= n_late;
    stats.workspace_in_use -= s.ws;
    s.reqs.clear();
    s.arr.clear();
    s.busy = false;
    s.ws = 0;
    cv_done.notify_all();
    return true;
}

bool gace_server::try_launch(ServeSlot& s, std::unique_lock<std::mutex>& lk) {
    if (s.busy || queue.empty()) return false;
    // admission: arrival order, while the estimated workspace fits the slot
    uint64_t ws = 0;
    while (!queue.empty() && s.reqs.size() < cfg.max_batch) {
        OwnedRequest& o = *queue.front();
        if (!s.reqs.empty() && ws + o.ws_est > slot_budget) break;
        ws += o.ws_est;
        s.reqs.push_back(std::move(queue.front()));
        queue.pop_front();
    }
    stats.queued = queue.size();
    stats.inflight += s.reqs.size();
    stats.batches += 1;
    stats.workspace_in_use += ws;
    if (stats.workspace_in_use > stats.workspace_peak) stats.workspace_peak = stats.workspace_in_use;
    s.ws = ws;
    s.busy = true;
    s.arr.clear();
    for (auto& o : s.reqs) s.arr.push_back(o->r);
    s.per.assign(s.arr.size(), GACE_OK);
    s.fin.assign(s.arr.size(), 0);
    s.ctx->zonemaps = zonemaps;
    lk.unlock();
    gace::CompileOptions opt;
    opt.item_rows = s.ctx->sched.item_rows;
    opt.join_part_keys = s.ctx->sched.join_part_keys;
    opt.workers = (uint32_t)s.ctx->n_cu * s.ctx->sched.wgs_per_cu;
    gace::compile_batch(s.arr.data(), (uint32_t)s.arr.size(), opt, s.cb);
    gace_status st = gace::apply_zonemaps(s.ctx, s.cb, s.arr.data(), s.stream);
    if (st == GACE_OK) st = gace::launch_compiled(s.ctx, s.cb, s.stream, true);
    lk.lock();
    if (st != GACE_OK) {
        const uint64_t t_done = now_ns();
        for (auto& o : s.reqs) {
            TicketState& t = tickets[o->ticket];
            t.done = true;
            t.st = st;
            t.done_ns = t_done;
        }
        stats.completed += s.reqs.size();
        stats.inflight -= s.reqs.size();
        stats.workspace_in_use -= s.ws;
        s.reqs.clear();
        s.busy = false;
        s.ws = 0;
        cv_done.notify_all();
    }
    return true;
}

void gace_server::run() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        bool progress = false;
        for (auto& s : slots) progress |= try_complete(s, lk);
        for (auto& s : slots) progress |= try_launch(s, lk);
        bool any_busy = false;
        for (auto& s : slots) any_busy |= s.busy;
        if (stop && queue.empty() && !any_busy) break;
        if (!progress) {
            if (any_busy) {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            } else {
                cv_work.wait_for(lk, std::chrono::milliseconds(50));
            }
        }
    }
}

using gace::set_error;

extern "C" {

gace_status gace_server_create(int hip_device, const gace_server_cfg* cfg, gace_server** out) {
    if (!cfg || !out || cfg->max_inflight < 1 || cfg->max_inflight > 8 || cfg->max_batch < 1 ||
        cfg->queue_capacity < 1 || (cfg->flags & ~GACE_SERVER_BATCH_COMPLETION)) {
        set_error("invalid server configuration");
        return GACE_EINVAL;
    }
    auto* srv = new gace_server();
    srv->cfg = *cfg;
    srv->device = hip_device;
    const uint64_t per = cfg->workspace_bytes / cfg->max_inflight;
    srv->slots.resize(cfg->max_inflight);
    for (auto& s : srv->slots) {
        gace_status st = gace_create(hip_device, per, &s.ctx);
        // requests finish as their scan or join does, unless asked otherwise
        if (st == GACE_OK) s.ctx->early = !(cfg->flags & GACE_SERVER_BATCH_COMPLETION);
        if (st == GACE_OK && hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess) {
            set_error("stream creation failed");
            st = GACE_EDEVICE;
        }
        if (st != GACE_OK) {
            for (auto& t : srv->slots) {
                if (t.stream) (void)hipStreamDestroy(t.stream);
                if (t.ctx) gace_destroy(t.ctx);
            }
            delete srv;
            return st;
        }
    }
    srv->slot_budget = srv->slots[0].ctx->arena_bytes;
    srv->worker = std::thread([srv] { srv->run(); });
    *out = srv;
    return GACE_OK;
}

gace_status gace_server_submit(gace_server* srv, const gace_request* req, uint64_t* ticket) {
    if (!srv || !req || !ticket) {
        set_error("NULL argument");
        return GACE_EINVAL;
    }
    std::string msg;
    gace_status st = gace::check_request(req, msg);
    if (st != GACE_OK) {
        std::lock_guard<std::mutex> g(srv->mu);
        srv->stats.rejected += 1;
        set_error(msg);
        return st;
    }
    auto o = std::make_unique<OwnedRequest>();
    o->r = *req;
    if (req->kind == GACE_REQ_SELECTIVITY) {
        o->cols.assign(req->table.cols, req->table.cols + req->table.n_cols);
        o->r.table.cols = o->cols.data();
        const uint32_t np = req->preds.n_preds;
        if (np) {
            o->pred_off.assign(req->preds.pred_off, req->preds.pred_off + np + 1);
            o->terms.assign(req->preds.terms, req->preds.terms + o->pred_off[np]);
        }
        o->r.preds.pred_off = o->pred_off.data();
        o->r.preds.terms = o->terms.data();
        o->ws_est = 0;
    }
    std::lock_guard<std::mutex> g(srv->mu);
    if (req->kind == GACE_REQ_JOIN) {
        o->ws_est = join_bytes(*req);
        if (o->ws_est > srv->slot_budget) {
            srv->stats.rejected += 1;
            set_error("request needs " + std::to_string(o->ws_est) + " workspace bytes; a slot has " +
                      std::to_string(srv->slot_budget));
            return GACE_ENOMEM;
        }
    }
    if (srv->queue.size() + srv->stats.inflight >= srv->cfg.queue_capacity) {
        set_error("server queue full");
        return GACE_EBUSY;
    }
    o->ticket = srv->next_ticket++;
    *ticket = o->ticket;
    TicketState ts;
    ts.submit_ns = now_ns();
    srv->tickets[o->ticket] = ts;
    srv->queue.push_back(std::move(o));
    srv->stats.submitted += 1;
    srv->stats.queued = srv->queue.size();
    srv->cv_work.notify_one();
    return GACE_OK;
}

gace_status gace_server_wait(gace_server* srv, uint64_t ticket, int64_t timeout_ns, gace_status* req_status) {
    return gace_server_wait_times(srv, ticket, timeout_ns, req_status, nullptr, nullptr);
}

gace_status gace_server_wait_times(gace_server* srv, uint64_t ticket, int64_t timeout_ns, gace_status* req_status,
                                   uint64_t* submit_ns, uint64_t* done_ns) {
    if (!srv) {
        set_error("NULL server");
        return GACE_EINVAL;
    }
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->tickets.find(ticket);
    if (it == srv->tickets.end()) {
        set_error("unknown ticket");
        return GACE_EINVAL;
    }
    // the ticket may be collected by another waiter meanwhile: never re-create it
    auto done = [&] {
        auto t = srv->tickets.find(ticket);
        return t == srv->tickets.end() || t->second.done;
    };
    if (timeout_ns < 0) {
        srv->cv_done.wait(lk, done);
    } else if (!srv->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), done)) {
        set_error("request still running");
        return GACE_ETIMEOUT;
    }
    it = srv->tickets.find(ticket);
    if (it == srv->tickets.end()) {
        set_error("ticket already collected by another wait");
        return GACE_EINVAL;
    }
    const TicketState& t = it->second;
    if (req_status) *req_status = t.st;
    if (submit_ns) *submit_ns = t.submit_ns;
    if (done_ns) *done_ns = t.done_ns;
    srv->tickets.erase(ticket);
    return GACE_OK;
}

gace_status gace_server_attach_zonemap(gace_server* srv, const gace_zonemap* zm) {
    if (!srv || !zm) {
        set_error("NULL argument");
        return GACE_EINVAL;
    }
    if (gace::zonemap_device(zm) != srv->device) {
        set_error("the zone map is on another device than the server");
        return GACE_EINVAL;
    }
    std::lock_guard<std::mutex> g(srv->mu);
    for (const gace_zonemap* z : srv->zonemaps)
        if (z == zm) return GACE_OK;
    srv->zonemaps.push_back(zm);
    return GACE_OK;
}

gace_status gace_server_stats_get(gace_server* srv, gace_server_stats* out) {
    if (!srv || !out) {
        set_error("NULL argument");
        return GACE_EINVAL;
    }
    std::lock_guard<std::mutex> g(srv->mu);
    *out = srv->stats;
    out->queued = srv->queue.size();
    return GACE_OK;
}

gace_status gace_server_destroy(gace_server* srv) {
    if (!srv) return GACE_OK;
    {
        std::lock_guard<std::mutex> g(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    if (srv->worker.joinable()) srv->worker.join();
    for (auto& s : srv->slots) {
        if (s.stream) (void)hipStreamDestroy(s.stream);
        if (s.ctx) gace_destroy(s.ctx);
    }
    delete srv;
    return GACE_OK;
}

}  // extern "C"
