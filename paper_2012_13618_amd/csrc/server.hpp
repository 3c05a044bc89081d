// Served form with continuous admission: requests arrive one by one and
// several workers, each with its own stream and device memory, serve them in
// runs that overlap on the device.  A free worker starts a run at once with
// the oldest queued requests: the first one, then the following ones while
// the run holds fewer than max_run_pins input pins (a large request runs
// nearly alone, small ones go together), at most max_slots requests, and
// while the footprint estimates of every run in flight stay within the
// budget; otherwise it waits until a run in flight ends.  So a request that
// arrives while others are on the device starts as soon as a worker and
// memory are free, and a small request never waits behind a large one that
// is already running.  A request whose own estimate is above the budget is
// refused at submission.  Each result is the partition the request gets
// alone (every run is the batched form, whose results equal the per-graph
// ones).
//
// Included once, from the library's C ABI translation unit.
#pragma once
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

namespace bp {

// Device bytes a partition of (N, E, P) with k parts holds at its peak: the
// per-tree-level working set (every coarsening level's CSR, incidence, sort
// buffers and scratch) times the number of tree levels, plus fixed state.
// The coefficients bound the measured use of the synthetic workloads with a
// margin (checked by a GPU test).
inline int64_t footprint_bytes(int64_t N, int64_t E, int64_t P, int32_t k)
{
    int64_t levels = 1;
    while (((int64_t)1 << levels) < (int64_t)k) levels++;
    // per tree level: the level stack of one bisection per segment (pins,
    // incidence, coarse hyperedges and their sort buffers dominate); measured
    // at 0.43-0.87 of this on netlist and column-net shapes of 0.1M-38M pins
    int64_t per = 384 * P + 128 * N + 96 * E;
    return levels * per + (int64_t(8) << 20);
}

struct Request {
    uint64_t ticket = 0;
    int32_t N = 0, E = 0, k = 2;
    double eps = 0.0;
    std::vector<int32_t> off, pins, nw, hw;
    bool has_nw = false, has_hw = false;
    int64_t footprint = 0;
    // result
    bool done = false;
    bp_status status = BP_OK;
    std::string error;
    std::vector<int32_t> part;
    BatchOut out;
    int32_t batch_size = 0;
    std::chrono::steady_clock::time_point t_submit, t_start, t_end;
};

struct Server {
    bp_server_config cfg{};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> tickets;
    uint64_t next_ticket = 1;
    int64_t queued_bytes = 0, queued_pins = 0;
    int64_t inflight_bytes = 0;  // footprint estimates of the runs on the device
    bool stop = false;
    int32_t waiters = 0;
    std::vector<std::thread> workers;

    // enough queued to start a run without waiting out the batching delay
    bool run_full() const
    {
        return (int32_t)queue.size() >= cfg.max_slots || queued_bytes >= cfg.hbm_budget_bytes ||
               queued_pins >= cfg.max_run_pins;
    }
    // the oldest queued request fits beside the runs in flight
    bool head_fits() const
    {
        return !queue.empty() && inflight_bytes + queue.front()->footprint <= cfg.hbm_budget_bytes;
    }
};

// Partitions the requests of one run; fills their results.
inline void serve_run(Server *s, Ctx &cx, std::vector<std::shared_ptr<Request>> &run)
{
    const int32_t n = (int32_t)run.size();
    std::vector<BatchItem> items(n);
    std::vector<int32_t *> outs(n);
    std::vector<int64_t> obase(n + 1, 0);
    for (int32_t i = 0; i < n; i++) obase[i + 1] = obase[i] + run[i]->N;
    int32_t *dpart = cx.ar->get<int32_t>(std::max<int64_t>(obase[n], 1));
    hipStream_t st = cx.lc.stream;
    for (int32_t i = 0; i < n; i++) {
        Request &r = *run[i];
        int64_t P = r.off[r.E];
        int32_t *off = cx.ar->get<int32_t>((int64_t)r.E + 1), *pins = cx.ar->get<int32_t>(P);
        BP_HIP(hipMemcpyAsync(off, r.off.data(), sizeof(int32_t) * r.off.size(), hipMemcpyHostToDevice, st));
        if (P > 0) BP_HIP(hipMemcpyAsync(pins, r.pins.data(), sizeof(int32_t) * P, hipMemcpyHostToDevice, st));
        int32_t *nw = nullptr, *hw = nullptr;
        if (r.has_nw) {
            nw = cx.ar->get<int32_t>(r.N);
            BP_HIP(hipMemcpyAsync(nw, r.nw.data(), sizeof(int32_t) * r.nw.size(), hipMemcpyHostToDevice, st));
        }
        if (r.has_hw) {
            hw = cx.ar->get<int32_t>(r.E);
            BP_HIP(hipMemcpyAsync(hw, r.hw.data(), sizeof(int32_t) * r.hw.size(), hipMemcpyHostToDevice, st));
        }
        items[i] = BatchItem{r.N, r.E, off, pins, nw, hw, r.k, r.eps};
        outs[i] = dpart + obase[i];
    }
    int32_t tl = 0;
    std::vector<BatchOut> res = partition_batch(cx, items, outs, &tl);
    std::vector<int32_t> host((size_t)obase[n]);
    if (obase[n] > 0)
        BP_HIP(hipMemcpyAsync(host.data(), dpart, sizeof(int32_t) * (size_t)obase[n], hipMemcpyDeviceToHost, st));
    BP_HIP(hipStreamSynchronize(st));
    for (int32_t i = 0; i < n; i++) {
        Request &r = *run[i];
        r.part.assign(host.begin() + obase[i], host.begin() + obase[i + 1]);
        r.out = res[i];
        r.status = res[i].balanced ? BP_OK : BP_WARN_IMBALANCED;
        r.batch_size = n;
    }
}

inline void serve_loop(Server *s)
{
    std::string init_error;
    hipStream_t stream = nullptr;
    LevelInfo *info_h = nullptr;
    Arena arena;
    if (hipSetDevice(s->cfg.device) != hipSuccess || hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess ||
        hipHostMalloc((void **)&info_h, 4096, hipHostMallocDefault) != hipSuccess) {
        init_error = std::string("server device setup failed: ") + hipGetErrorString(hipGetLastError());
    }
    for (;;) {
        std::vector<std::shared_ptr<Request>> run;
        int64_t run_bytes = 0;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stop || s->head_fits(); });
            if (s->stop) break;
            if (s->cfg.max_batch_delay_us > 0 && !s->run_full()) {
                auto until = s->queue.front()->t_submit + std::chrono::microseconds(s->cfg.max_batch_delay_us);
                s->cv_work.wait_until(lk, until, [&] { return s->stop || s->run_full(); });
                if (s->stop) break;
                if (!s->head_fits()) continue;  // another worker took the requests meanwhile
            }
            int64_t pins = 0;
            while (!s->queue.empty() && (int32_t)run.size() < s->cfg.max_slots &&
                   (run.empty() || pins + (int64_t)s->queue.front()->pins.size() <= s->cfg.max_run_pins) &&
                   s->inflight_bytes + run_bytes + s->queue.front()->footprint <= s->cfg.hbm_budget_bytes) {
                auto &r = s->queue.front();
                run_bytes += r->footprint;
                pins += (int64_t)r->pins.size();
                s->queued_bytes -= r->footprint;
                s->queued_pins -= (int64_t)r->pins.size();
                run.push_back(r);
                s->queue.pop_front();
            }
            s->inflight_bytes += run_bytes;
        }
        // more queued requests may fit beside this run on another worker
        s->cv_work.notify_one();
        auto t0 = std::chrono::steady_clock::now();
        for (auto &r : run) r->t_start = t0;
        bp_status err = BP_OK;
        std::string msg;
        try {
            if (!init_error.empty()) throw Error(BP_ERR_DEVICE, init_error);
            arena.reset();
            Ctx cx;
            cx.ar = &arena;
            cx.info_h = info_h;
            cx.info_d = arena.get<LevelInfo>(1);
            cx.lc.stream = stream;
            cx.prm = s->cfg.params;
            serve_run(s, cx, run);
        } catch (const Error &e) {
            err = e.status;
            msg = e.what();
        } catch (const std::exception &e) {
            err = BP_ERR_DEVICE;
            msg = e.what();
        }
        auto t1 = std::chrono::steady_clock::now();
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->inflight_bytes -= run_bytes;
            for (auto &r : run) {
                if (err != BP_OK) {
                    r->status = err;
                    r->error = msg;
                }
                r->t_end = t1;
                r->done = true;
            }
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();  // memory freed: a waiting worker may start
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto &r : s->queue) {
            r->status = BP_ERR_SHUTDOWN;
            r->error = "server destroyed before the request ran";
            r->t_end = std::chrono::steady_clock::now();
            r->done = true;
        }
        s->queue.clear();
        s->queued_bytes = 0;
        s->queued_pins = 0;
    }
    s->cv_done.notify_all();
    if (stream) (void)hipStreamSynchronize(stream);
    arena.release();
    if (info_h) (void)hipHostFree(info_h);
    if (stream) (void)hipStreamDestroy(stream);
}

}  // namespace bp

struct bp_server {
    bp::Server s;
};

extern "C" {

void bp_server_default_config(bp_server_config *c)
{
    if (!c) return;
    c->hbm_budget_bytes = int64_t(64) << 30;
    c->max_slots = 256;
    c->max_batch_delay_us = 0;
    c->device = 0;
    c->workers = 4;
    bp_default_params(&c->params);
    c->max_run_pins = int64_t(4) << 20;
}

bp_status bp_request_footprint(int32_t num_nodes, int32_t num_hedges, int64_t num_pins, int32_t k,
                               int64_t *bytes)
{
    if (num_nodes < 0 || num_hedges < 0 || num_pins < 0 || k < 1 || !bytes)
        return fail(BP_ERR_INVALID_ARG, "bad footprint arguments");
    *bytes = bp::footprint_bytes(num_nodes, num_hedges, num_pins, k);
    return BP_OK;
}

bp_status bp_server_create(const bp_server_config *cfg, bp_server **out)
{
    if (!cfg || !out) return fail(BP_ERR_INVALID_ARG, "NULL config or output");
    if (cfg->hbm_budget_bytes <= 0 || cfg->max_slots < 1 || cfg->max_batch_delay_us < 0 || cfg->device < 0 ||
        cfg->workers < 1 || cfg->workers > 16 || cfg->max_run_pins < 1)
        return fail(BP_ERR_INVALID_ARG, "invalid server config");
    bp_status st = check_params(&cfg->params);
    if (st != BP_OK) return st;
    BP_GUARD_BEGIN
    bp_server *srv = new bp_server();
    srv->s.cfg = *cfg;
    for (int32_t w = 0; w < cfg->workers; w++) srv->s.workers.emplace_back(bp::serve_loop, &srv->s);
    *out = srv;
    return BP_OK;
    BP_GUARD_END
}

bp_status bp_server_submit(bp_server *srv, const bp_hypergraph *hg, int32_t k, double eps, uint64_t *ticket)
{
    if (!srv || !ticket) return fail(BP_ERR_INVALID_ARG, "NULL server or ticket");
    bp_status st = validate_host(hg);
    if (st != BP_OK) return st;
    if (k < 1 || !(eps >= 0.0) || std::isinf(eps)) return fail(BP_ERR_INVALID_ARG, "k < 1 or bad eps");
    bp::Server &s = srv->s;
    int64_t P = hg->hedge_offsets[hg->num_hedges];
    int64_t fp = bp::footprint_bytes(hg->num_nodes, hg->num_hedges, P, k);
    if (fp > s.cfg.hbm_budget_bytes)
        return fail(BP_ERR_REJECTED, "request needs about " + std::to_string(fp) + " device bytes, budget is " +
                                         std::to_string(s.cfg.hbm_budget_bytes));
    BP_GUARD_BEGIN
    auto r = std::make_shared<bp::Request>();
    r->N = hg->num_nodes;
    r->E = hg->num_hedges;
    r->k = k;
    r->eps = eps;
    r->footprint = fp;
    r->off.assign(hg->hedge_offsets, hg->hedge_offsets + hg->num_hedges + 1);
    if (P > 0) r->pins.assign(hg->pins, hg->pins + P);
    if ((r->has_nw = hg->node_weights != nullptr)) r->nw.assign(hg->node_weights, hg->node_weights + r->N);
    if ((r->has_hw = hg->hedge_weights != nullptr)) r->hw.assign(hg->hedge_weights, hg->hedge_weights + r->E);
    r->t_submit = std::chrono::steady_clock::now();
    {
        std::lock_guard<std::mutex> lk(s.mu);
        if (s.stop) return fail(BP_ERR_SHUTDOWN, "server is shutting down");
        r->ticket = s.next_ticket++;
        s.tickets[r->ticket] = r;
        s.queue.push_back(r);
        s.queued_bytes += fp;
        s.queued_pins += P;
        *ticket = r->ticket;
    }
    s.cv_work.notify_one();
    return BP_OK;
    BP_GUARD_END
}

bp_status bp_server_wait(bp_server *srv, uint64_t ticket, int32_t *part_out, int64_t *cut_out,
                         bp_req_stats *stats)
{
    if (!srv) return fail(BP_ERR_INVALID_ARG, "NULL server");
    bp::Server &s = srv->s;
    std::shared_ptr<bp::Request> r;
    {
        std::unique_lock<std::mutex> lk(s.mu);
        auto it = s.tickets.find(ticket);
        if (it == s.tickets.end()) return fail(BP_ERR_NOT_FOUND, "unknown or already collected ticket");
        r = it->second;
        s.waiters++;
        s.cv_done.wait(lk, [&] { return r->done; });
        s.waiters--;
        s.tickets.erase(ticket);
    }
    s.cv_done.notify_all();
    if (r->status < 0) return fail(r->status, r->error);
    if (r->N > 0 && part_out) std::memcpy(part_out, r->part.data(), sizeof(int32_t) * (size_t)r->N);
    if (cut_out) *cut_out = r->out.cut;
    if (stats) {
        using ms = std::chrono::duration<double, std::milli>;
        stats->cut = r->out.cut;
        stats->max_part_weight = r->out.maxw;
        stats->part_weight_limit = r->out.limit;
        stats->balanced = r->out.balanced;
        stats->batch_size = r->batch_size;
        stats->footprint_bytes = r->footprint;
        stats->queue_ms = ms(r->t_start - r->t_submit).count();
        stats->run_ms = ms(r->t_end - r->t_start).count();
        stats->latency_ms = ms(r->t_end - r->t_submit).count();
    }
    return r->status;
}

bp_status bp_server_destroy(bp_server *srv)
{
    if (!srv) return fail(BP_ERR_INVALID_ARG, "NULL server");
    bp::Server &s = srv->s;
    {
        std::lock_guard<std::mutex> lk(s.mu);
        s.stop = true;
    }
    s.cv_work.notify_all();
    for (auto &w : s.workers)
        if (w.joinable()) w.join();
    {
        std::unique_lock<std::mutex> lk(s.mu);
        s.cv_done.wait(lk, [&] { return s.waiters == 0; });
    }
    delete srv;
    return BP_OK;
}

}  // extern "C"
