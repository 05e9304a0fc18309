// qt_server.cpp -- continuous-batching request server.
//
// Requests (one batch each) are queued by qt_submit.  A scheduler thread runs
// rounds: at each round boundary it admits queued requests, in arrival
// order, while their device memory fits the HBM budget and their
// trajectories fit the device's resident slots (times max_occupancy: slots
// kept busy, the queue taking the excess instead of every running request
// slowing down), then runs every unfinished trajectory of
// every admitted request for up to segment_steps steps, in one persistent
// launch per grid size N (trajectories of different requests share the
// launch and refill the same workgroups; the launches of the grid sizes
// run concurrently), and retires finished requests:
// their results are copied to host memory, their device memory is freed and
// their latency (completion - submission) is recorded.  A trajectory's
// result depends only on its own inputs and ids and on the kernel variant,
// which the server fixes per (N, potential) at its first use and keeps for
// its life (later qt_plan calls on the context do not change it), so a
// request gives bitwise the same result alone or in a mix.  A request whose
// admission or result copy fails ends with that failure's status.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <thread>
#include <vector>

#include "qt_host.hpp"

using namespace qt;
using Clock = std::chrono::steady_clock;

namespace {

enum ReqState { QUEUED, RUNNING, DONE, CANCELED, FAILED };

struct Request {
    uint64_t id = 0;
    HostBatch hb;
    ReqState state = QUEUED;
    Clock::time_point t_submit, t_done;
    bool cancel = false;
    // device side while running
    DeviceGroups dg;
    ResultBuffers res;
    TrajState* st = nullptr;
    void* st_psi = nullptr;
    size_t bytes = 0;
    double occ = 0.0;             // its trajectories per resident slot
    // host results once done
    std::vector<double> norm, first_r, overlap, survival, mean_r, min_gap;
    std::vector<int32_t> l, color, n_jumps, status;
    std::vector<int64_t> steps_done;
    std::vector<char> psi_raw;    // final wave functions, kernel precision
    // FAILED: the status and message of the failure
    qt_status fail_status = QT_OK;
    std::string fail_msg;
};

// The kernel variant of one (N, potential) class, fixed at its first use.
struct Variant {
    int W = 0, slots = 0;
    fused_launcher launch = nullptr;
};

}  // namespace

struct qt_server {
    qt_context* ctx = nullptr;
    qt_server_cfg cfg{};
    size_t budget = 0, in_use = 0;
    double max_occ = 8.0, occ = 0.0;   // admitted trajectories per resident slot
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> queue;
    std::map<uint64_t, std::shared_ptr<Request>> all;
    std::vector<std::shared_ptr<Request>> running;
    uint64_t next_id = 1;
    bool stop = false;
    std::thread th;
    hipStream_t stream = nullptr;
    void* misc = nullptr;
    size_t misc_bytes = 0;
    std::vector<double> latencies;
    int64_t completed = 0, admitted = 0, traj_steps = 0;
    double busy_s = 0.0;
    std::string error;
    std::map<int, Variant> variants;   // by 2 N + potential
    // fork streams of the concurrent per-N launches of a round
    std::vector<hipStream_t> fork_streams;
    std::vector<hipEvent_t> fork_joins;
    hipEvent_t fork = nullptr;
};

namespace {

size_t request_bytes(const HostBatch& hb, int prec)
{
    const int64_t n = std::max<int64_t>(hb.batch.n_traj, 1);
    const size_t state = n * sizeof(TrajState) + (size_t)n * hb.phys.N * elem_bytes(prec);
    const size_t tables = 16 * (size_t)hb.phys.N * 8 + hb.tau.size() * 16 + 4096;
    return state + result_bytes(n) + tables + (size_t)n * 12;
}

qt_status admit(qt_server* s, Request& q)
{
    const int prec = s->cfg.precision;
    const int64_t n = std::max<int64_t>(q.hb.batch.n_traj, 1);
    qt_status st = alloc_results(q.hb.batch.n_traj, &q.res);
    if (st != QT_OK) return st;
    if (hipMalloc(reinterpret_cast<void**>(&q.st), n * sizeof(TrajState)) != hipSuccess ||
        hipMalloc(&q.st_psi, (size_t)n * q.hb.phys.N * elem_bytes(prec)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(QT_ENOMEM, "no device memory for the state of %lld trajectories",
                    (long long)n);
    }
    QT_HIP(hipMemsetAsync(q.st, 0, n * sizeof(TrajState), s->stream));
    std::vector<const HostBatch*> hbv{&q.hb};
    std::vector<qt_results> outs{q.res.r};
    {
        std::lock_guard<std::mutex> lk(s->ctx->mu);   // the context's table caches
        std::vector<HostBatch*> hv{&q.hb};
        if ((st = run_vacuum_phases(s->ctx, hv, prec, s->stream)) != QT_OK) return st;
        if ((st = upload_groups(s->ctx, hbv, prec, outs, false, s->stream, false, &q.dg)) != QT_OK)
            return st;
    }
    q.dg.host[0].st = q.st;
    q.dg.host[0].st_psi = q.st_psi;
    q.state = RUNNING;
    return QT_OK;
}

void release(Request& q)
{
    hipFree(q.res.mem);
    hipFree(q.st);
    hipFree(q.st_psi);
    hipFree(q.dg.mem);
    q.res.mem = q.st = nullptr;
    q.st_psi = q.dg.mem = nullptr;
}

// The kernel variant of (N, potential), fixed at its first use.
qt_status server_variant(qt_server* s, int N, int pot, Variant** out)
{
    Variant& v = s->variants[2 * N + pot];
    if (!v.launch) {
        std::lock_guard<std::mutex> lk(s->ctx->mu);
        qt_status st = pick_launcher(s->ctx, s->cfg.precision, N, pot, &v.W, &v.launch, &v.slots);
        if (st != QT_OK) return st;
    }
    *out = &v;
    return QT_OK;
}

// Marks q failed with the calling thread's last error (the caller holds s->mu).
void mark_failed(Request& q, qt_status st)
{
    q.state = FAILED;
    q.fail_status = st;
    q.fail_msg = qt_last_error();
}

qt_status fetch_results(qt_server* s, Request& q)
{
    const int64_t n = q.hb.batch.n_traj;
    q.norm.resize(n); q.first_r.resize(n); q.overlap.resize(6 * n); q.survival.resize(6 * n);
    q.mean_r.resize(n); q.min_gap.resize(n); q.l.resize(n); q.color.resize(n);
    q.n_jumps.resize(n); q.status.resize(n); q.steps_done.resize(n);
    qt_results h{};
    h.norm = q.norm.data(); h.first_r = q.first_r.data(); h.overlap = q.overlap.data();
    h.survival = q.survival.data(); h.mean_r = q.mean_r.data(); h.min_gap = q.min_gap.data();
    h.l = q.l.data(); h.color = q.color.data(); h.n_jumps = q.n_jumps.data();
    h.status = q.status.data(); h.steps_done = q.steps_done.data();
    qt_status st = copy_results(q.res.r, h, n, hipMemcpyDeviceToHost, s->stream);
    if (st != QT_OK) return st;
    // final wave functions (kept in the checkpoint buffer) in the kernel's
    // precision; widened to FP64 on the host by qt_wait when asked for
    q.psi_raw.resize((size_t)n * q.hb.phys.N * elem_bytes(s->cfg.precision));
    if (n)
        QT_HIP(hipMemcpyAsync(q.psi_raw.data(), q.st_psi, q.psi_raw.size(), hipMemcpyDeviceToHost,
                              s->stream));
    QT_HIP(hipStreamSynchronize(s->stream));
    return QT_OK;
}

// One round over the running requests.  Returns the number of
// trajectory-steps it advanced.
qt_status run_round(qt_server* s, int64_t* advanced)
{
    *advanced = 0;
    const int prec = s->cfg.precision;
    std::vector<GroupDesc> groups;
    std::vector<int> gN;
    for (auto& q : s->running) {
        groups.push_back(q->dg.host[0]);
        gN.push_back(2 * q->hb.phys.N + q->hb.phys.potential);
    }
    // items of every running request, grouped by (N, potential) (keyed
    // 2 N + potential: the kernels are specialised on both)
    std::vector<int> Ns;
    for (int N : gN)
        if (std::find(Ns.begin(), Ns.end(), N) == Ns.end()) Ns.push_back(N);
    size_t n_items = 0;
    for (auto& q : s->running) n_items += (size_t)q->hb.batch.n_traj;
    const size_t need = 256 + ((groups.size() * sizeof(GroupDesc) + 255) & ~(size_t)255) +
                        ((n_items * 4 + 255) & ~(size_t)255) + n_items * 8 + 256;
    if (need > s->misc_bytes) {
        if (s->misc) QT_HIP(hipFree(s->misc));
        s->misc_bytes = need * 2;
        QT_HIP(hipMalloc(&s->misc, s->misc_bytes));
    }
    char* m = static_cast<char*>(s->misc);
    int32_t* queues = reinterpret_cast<int32_t*>(m);
    GroupDesc* dgroups = reinterpret_cast<GroupDesc*>(m + 256);
    int32_t* ig = reinterpret_cast<int32_t*>(m + 256 + ((groups.size() * sizeof(GroupDesc) + 255) & ~(size_t)255));
    int64_t* ii = reinterpret_cast<int64_t*>(reinterpret_cast<char*>(ig) + ((n_items * 4 + 255) & ~(size_t)255));
    std::vector<int32_t> hig;
    std::vector<int64_t> hii;
    std::vector<size_t> start, count;
    for (int N : Ns) {
        start.push_back(hig.size());
        for (size_t g = 0; g < s->running.size(); ++g) {
            if (gN[g] != N) continue;
            for (int64_t i = 0; i < s->running[g]->hb.batch.n_traj; ++i) {
                hig.push_back((int32_t)g);
                hii.push_back(i);
            }
        }
        count.push_back(hig.size() - start.back());
    }
    QT_HIP(hipMemcpyAsync(dgroups, groups.data(), groups.size() * sizeof(GroupDesc), hipMemcpyHostToDevice, s->stream));
    if (n_items) {
        QT_HIP(hipMemcpyAsync(ig, hig.data(), n_items * 4, hipMemcpyHostToDevice, s->stream));
        QT_HIP(hipMemcpyAsync(ii, hii.data(), n_items * 8, hipMemcpyHostToDevice, s->stream));
    }
    std::vector<ClassLaunch> cl;
    for (size_t c = 0; c < Ns.size(); ++c) {
        if (!count[c]) continue;
        const int N = Ns[c] / 2, pot = Ns[c] % 2;
        qt_context::Tables t;
        qt_status st;
        Variant* v = nullptr;
        if ((st = server_variant(s, N, pot, &v)) != QT_OK) return st;
        {
            std::lock_guard<std::mutex> lk(s->ctx->mu);
            if ((st = ensure_tables(s->ctx, prec, N, &t)) != QT_OK) return st;
        }
        const fused_launcher launch = v->launch;
        const int slots = v->slots;
        FusedArgs a;
        a.groups = dgroups;
        a.item_group = ig + start[c];
        a.item_index = ii + start[c];
        a.n_items = (int32_t)count[c];
        a.queue = queues + c;
        a.tw = t.tw;
        a.prew = t.prew;
        a.seg_steps = s->cfg.segment_steps;
        const int grid = (int)std::min<int64_t>((int64_t)count[c], (int64_t)s->ctx->n_cu * slots);
        cl.push_back(ClassLaunch{launch, a, grid});
    }
    // the N classes of the round run concurrently (see launch_classes)
    if (qt_status st = launch_classes(cl, s->stream, &s->fork, &s->fork_streams, &s->fork_joins);
        st != QT_OK)
        return st;
    QT_HIP(hipStreamSynchronize(s->stream));
    // progress: read the state records back
    for (auto& q : s->running) {
        const int64_t n = q->hb.batch.n_traj;
        std::vector<TrajState> h((size_t)n);
        if (n) QT_HIP(hipMemcpy(h.data(), q->st, n * sizeof(TrajState), hipMemcpyDeviceToHost));
        int64_t done = 0, steps = 0;
        for (const TrajState& t : h) {
            done += t.done;
            steps += t.step;
        }
        *advanced += steps;   // cumulative steps; the caller differences them
        if (done == n) q->state = DONE;
    }
    return QT_OK;
}

void server_loop(qt_server* s)
{
    hipSetDevice(s->ctx->device);
    std::map<uint64_t, int64_t> last_steps;
    while (true) {
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty() || !s->running.empty(); });
            if (s->stop) break;
            // drop cancelled running requests
            for (auto it = s->running.begin(); it != s->running.end();) {
                if ((*it)->cancel) {
                    release(**it);
                    s->in_use -= (*it)->bytes;
                    s->occ -= (*it)->occ;
                    (*it)->state = CANCELED;
                    it = s->running.erase(it);
                } else {
                    ++it;
                }
            }
            // admission in arrival order, by HBM budget and resident slots
            while (!s->queue.empty()) {
                auto q = s->queue.front();
                if (q->cancel) {
                    q->state = CANCELED;
                    s->queue.pop_front();
                    continue;
                }
                const size_t b = request_bytes(q->hb, s->cfg.precision);
                Variant* v = nullptr;
                const qt_status vst = server_variant(s, q->hb.phys.N, q->hb.phys.potential, &v);
                if (vst != QT_OK) {
                    s->queue.pop_front();
                    mark_failed(*q, vst);
                    continue;
                }
                const double o = (double)q->hb.batch.n_traj /
                                 ((double)s->ctx->n_cu * std::max(v->slots, 1));
                if (!s->running.empty() &&
                    (s->in_use + b > s->budget || (s->max_occ > 0 && s->occ + o > s->max_occ)))
                    break;
                s->queue.pop_front();
                q->bytes = b;
                q->occ = o;
                const qt_status ast = admit(s, *q);
                if (ast != QT_OK) {
                    // this request fails with the cause; the others go on
                    mark_failed(*q, ast);
                    release(*q);
                    continue;
                }
                s->in_use += b;
                s->occ += o;
                s->admitted++;
                s->running.push_back(q);
            }
            s->cv_done.notify_all();
        }
        if (s->running.empty()) continue;
        const auto t0 = Clock::now();
        int64_t adv = 0;
        qt_status st = run_round(s, &adv);
        const double dt = std::chrono::duration<double>(Clock::now() - t0).count();
        std::lock_guard<std::mutex> lk(s->mu);
        s->busy_s += dt;
        if (st != QT_OK) {
            // a failed round: every running request ends with its cause
            s->error = qt_last_error();
            for (auto& q : s->running) {
                release(*q);
                mark_failed(*q, st);
            }
            s->running.clear();
            s->in_use = 0;
            s->occ = 0.0;
            s->cv_done.notify_all();
            continue;
        }
        int64_t delta = 0;
        for (auto it = s->running.begin(); it != s->running.end();) {
            auto q = *it;
            // steps advanced by this request this round
            int64_t cur = 0;
            {
                const int64_t n = q->hb.batch.n_traj;
                std::vector<TrajState> h((size_t)n);
                if (n) hipMemcpy(h.data(), q->st, n * sizeof(TrajState), hipMemcpyDeviceToHost);
                for (const TrajState& t : h) cur += t.step;
            }
            delta += cur - last_steps[q->id];
            last_steps[q->id] = cur;
            if (q->state == DONE) {
                const qt_status fst = fetch_results(s, *q);
                if (fst != QT_OK) mark_failed(*q, fst);
                release(*q);
                s->in_use -= q->bytes;
                s->occ -= q->occ;
                q->t_done = Clock::now();
                s->latencies.push_back(std::chrono::duration<double>(q->t_done - q->t_submit).count());
                s->completed++;
                last_steps.erase(q->id);
                it = s->running.erase(it);
            } else {
                ++it;
            }
        }
        (void)adv;
        s->traj_steps += delta;
        if (trace_on())
            trace_line("{\"event\": \"round\", \"running\": %zu, \"queued\": %zu, "
                       "\"occupancy\": %.3f, \"traj_steps\": %lld, \"wall_ms\": %.3f}",
                       s->running.size(), s->queue.size(), s->occ, (long long)delta, dt * 1e3);
        s->cv_done.notify_all();
    }
}

}  // namespace

extern "C" {

qt_status qt_server_create(qt_context* ctx, const qt_server_cfg* cfg, qt_server** out)
{
    if (!ctx || !cfg || !out) return fail(QT_EINVAL, "null argument");
    if (cfg->segment_steps < 1) return fail(QT_EINVAL, "segment_steps must be >= 1");
    if (cfg->precision != QT_FP64 && cfg->precision != QT_FP32_BULK) return fail(QT_EINVAL, "bad precision");
    if (!std::isfinite(cfg->max_occupancy)) return fail(QT_EINVAL, "max_occupancy must be finite");
    QT_HIP(hipSetDevice(ctx->device));
    auto* s = new qt_server();
    s->ctx = ctx;
    s->cfg = *cfg;
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        delete s;
        return fail(QT_EDEVICE, "hipMemGetInfo failed");
    }
    s->budget = cfg->hbm_budget_bytes ? cfg->hbm_budget_bytes : fr / 2;
    s->max_occ = cfg->max_occupancy == 0.0 ? 8.0 : cfg->max_occupancy;
    if (hipStreamCreate(&s->stream) != hipSuccess) {
        delete s;
        return fail(QT_EDEVICE, "hipStreamCreate failed");
    }
    s->th = std::thread(server_loop, s);
    *out = s;
    return QT_OK;
}

qt_status qt_submit(qt_server* s, const qt_physics* phys, const qt_ttable* tt, const qt_init* init,
                    const qt_batch* batch, uint64_t* request_id)
{
    if (!s || !request_id) return fail(QT_EINVAL, "null argument");
    auto q = std::make_shared<Request>();
    qt_status st = prepare(s->ctx, phys, tt, init, batch, &q->hb);
    if (st != QT_OK) return st;
    if (batch->no_jump_shortcut) return fail(QT_EINVAL, "the no-jump shortcut is not available in the server");
    if (batch->precision != s->cfg.precision) return fail(QT_EINVAL, "request precision differs from the server's");
    if (batch->form != QT_FORM_FUSED) return fail(QT_EINVAL, "the server runs the fused form");
    if (request_bytes(q->hb, s->cfg.precision) > s->budget)
        return fail(QT_ENOMEM, "request needs %zu bytes, more than the HBM budget %zu",
                    request_bytes(q->hb, s->cfg.precision), s->budget);
    q->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    q->id = s->next_id++;
    s->all[q->id] = q;
    s->queue.push_back(q);
    *request_id = q->id;
    s->cv_work.notify_all();
    return QT_OK;
}

qt_status qt_poll(qt_server* s, uint64_t id, int32_t* done)
{
    if (!s || !done) return fail(QT_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(id);
    if (it == s->all.end()) return fail(QT_ENOTFOUND, "unknown request %llu", (unsigned long long)id);
    const ReqState rs = it->second->state;
    *done = rs == DONE || rs == CANCELED || rs == FAILED;
    return QT_OK;
}

qt_status qt_wait(qt_server* s, uint64_t id, const qt_results* host_out, double timeout_s)
{
    if (!s) return fail(QT_EINVAL, "null argument");
    if (host_out && host_out->jump_log) return fail(QT_EINVAL, "the server keeps no jump log");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(id);
    if (it == s->all.end()) return fail(QT_ENOTFOUND, "unknown request %llu", (unsigned long long)id);
    auto q = it->second;
    auto pred = [&] { return q->state == DONE || q->state == CANCELED || q->state == FAILED; };
    if (timeout_s < 0) {
        s->cv_done.wait(lk, pred);
    } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) {
        return fail(QT_ETIMEOUT, "request %llu not finished", (unsigned long long)id);
    }
    if (q->state == CANCELED) {
        s->all.erase(id);
        return fail(QT_ECANCELED, "request %llu was cancelled", (unsigned long long)id);
    }
    if (q->state == FAILED) {
        const qt_status st = q->fail_status;
        const std::string msg = q->fail_msg;
        s->all.erase(id);
        return fail(st, "request %llu failed: %s", (unsigned long long)id, msg.c_str());
    }
    if (host_out) {
        const size_t n = q->norm.size();
        auto cp = [&](void* d, const void* src, size_t b) { if (d && b) std::memcpy(d, src, b); };
        cp(host_out->norm, q->norm.data(), n * 8);
        cp(host_out->first_r, q->first_r.data(), n * 8);
        cp(host_out->overlap, q->overlap.data(), 6 * n * 8);
        cp(host_out->survival, q->survival.data(), 6 * n * 8);
        cp(host_out->mean_r, q->mean_r.data(), n * 8);
        cp(host_out->min_gap, q->min_gap.data(), n * 8);
        cp(host_out->l, q->l.data(), n * 4);
        cp(host_out->color, q->color.data(), n * 4);
        cp(host_out->n_jumps, q->n_jumps.data(), n * 4);
        cp(host_out->status, q->status.data(), n * 4);
        cp(host_out->steps_done, q->steps_done.data(), n * 8);
        if (host_out->psi) {
            const size_t cnt = (size_t)n * q->hb.phys.N;
            if (s->cfg.precision == QT_FP64) {
                cp(host_out->psi, q->psi_raw.data(), cnt * 16);
            } else {
                const float* f = reinterpret_cast<const float*>(q->psi_raw.data());
                for (size_t k = 0; k < 2 * cnt; ++k) host_out->psi[k] = (double)f[k];
            }
        }
    }
    s->all.erase(id);
    return QT_OK;
}

qt_status qt_cancel(qt_server* s, uint64_t id)
{
    if (!s) return fail(QT_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(id);
    if (it == s->all.end()) return fail(QT_ENOTFOUND, "unknown request %llu", (unsigned long long)id);
    it->second->cancel = true;
    s->cv_work.notify_all();
    return QT_OK;
}

qt_status qt_server_stats(qt_server* s, qt_stats* out)
{
    if (!s || !out) return fail(QT_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(out, 0, sizeof *out);
    std::vector<double> v = s->latencies;
    std::sort(v.begin(), v.end());
    if (!v.empty()) {
        auto pct = [&](double p) {
            const double x = p * (v.size() - 1);
            const size_t i = (size_t)x;
            const double f = x - i;
            return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
        };
        out->p50_latency_s = pct(0.50);
        out->p99_latency_s = pct(0.99);
        double sum = 0;
        for (double x : v) sum += x;
        out->mean_latency_s = sum / v.size();
    }
    out->traj_steps = s->traj_steps;
    out->traj_steps_per_s = s->busy_s > 0 ? s->traj_steps / s->busy_s : 0.0;
    out->completed = s->completed;
    out->admitted = s->admitted;
    out->queued = (int64_t)s->queue.size();
    out->running = (int64_t)s->running.size();
    out->hbm_in_use = s->in_use;
    return QT_OK;
}

qt_status qt_server_destroy(qt_server* s)
{
    if (!s) return QT_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->th.joinable()) s->th.join();
    hipSetDevice(s->ctx->device);
    for (auto& q : s->running) release(*q);
    if (s->misc) hipFree(s->misc);
    for (hipStream_t a : s->fork_streams) hipStreamDestroy(a);
    for (hipEvent_t e : s->fork_joins) hipEventDestroy(e);
    if (s->fork) hipEventDestroy(s->fork);
    if (s->stream) hipStreamDestroy(s->stream);
    delete s;
    return QT_OK;
}

}  // extern "C"
