// qt_job.cpp -- segmented runs: per-trajectory state in HBM between
// segments (the checkpoint), HIP-graph replay of the segment launches, save
// and restore of the whole state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <vector>

#include "qt_host.hpp"

namespace qt {

static size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

size_t result_bytes(int64_t n)
{
    const size_t d = (size_t)n * 8;
    return al(d) * 3 + al(6 * d) * 2 + al(d) + al((size_t)n * 4) * 4 + al(d) + al(d);
}

qt_status alloc_results(int64_t n, ResultBuffers* rb)
{
    rb->bytes = result_bytes(std::max<int64_t>(n, 1));
    QT_HIP(hipMalloc(&rb->mem, rb->bytes));
    char* p = static_cast<char*>(rb->mem);
    const size_t d = (size_t)std::max<int64_t>(n, 1) * 8;
    auto take = [&](size_t b) { char* q = p; p += al(b); return q; };
    rb->r.norm = reinterpret_cast<double*>(take(d));
    rb->r.first_r = reinterpret_cast<double*>(take(d));
    rb->r.mean_r = reinterpret_cast<double*>(take(d));
    rb->r.overlap = reinterpret_cast<double*>(take(6 * d));
    rb->r.survival = reinterpret_cast<double*>(take(6 * d));
    rb->r.min_gap = reinterpret_cast<double*>(take(d));
    const size_t i4 = (size_t)std::max<int64_t>(n, 1) * 4;
    rb->r.l = reinterpret_cast<int32_t*>(take(i4));
    rb->r.color = reinterpret_cast<int32_t*>(take(i4));
    rb->r.n_jumps = reinterpret_cast<int32_t*>(take(i4));
    rb->r.status = reinterpret_cast<int32_t*>(take(i4));
    rb->r.steps_done = reinterpret_cast<int64_t*>(take(d));
    rb->r.psi = nullptr;
    return QT_OK;
}

// Copies results (device buffers) to `dst` pointers of kind `kind`.
qt_status copy_results(const qt_results& src, const qt_results& dst, int64_t n, hipMemcpyKind kind,
                       hipStream_t s)
{
    if (n <= 0) return QT_OK;
    auto cp = [&](void* d, const void* sp, size_t b) -> qt_status {
        if (d && sp) QT_HIP(hipMemcpyAsync(d, sp, b, kind, s));
        return QT_OK;
    };
    const size_t d = (size_t)n * 8, i4 = (size_t)n * 4;
    qt_status st;
    if ((st = cp(dst.norm, src.norm, d)) != QT_OK) return st;
    if ((st = cp(dst.first_r, src.first_r, d)) != QT_OK) return st;
    if ((st = cp(dst.mean_r, src.mean_r, d)) != QT_OK) return st;
    if ((st = cp(dst.overlap, src.overlap, 6 * d)) != QT_OK) return st;
    if ((st = cp(dst.survival, src.survival, 6 * d)) != QT_OK) return st;
    if ((st = cp(dst.min_gap, src.min_gap, d)) != QT_OK) return st;
    if ((st = cp(dst.l, src.l, i4)) != QT_OK) return st;
    if ((st = cp(dst.color, src.color, i4)) != QT_OK) return st;
    if ((st = cp(dst.n_jumps, src.n_jumps, i4)) != QT_OK) return st;
    if ((st = cp(dst.status, src.status, i4)) != QT_OK) return st;
    if ((st = cp(dst.steps_done, src.steps_done, d)) != QT_OK) return st;
    return QT_OK;
}

}  // namespace qt

using namespace qt;

struct qt_job {
    qt_context* ctx = nullptr;
    int prec = 0, N = 0, W = 0;
    int64_t n_traj = 0, seg_steps = 0, n_steps = 0;
    HostBatch hb;
    DeviceGroups dg;
    ResultBuffers res;
    TrajState* st = nullptr;
    void* st_psi = nullptr;
    void* misc = nullptr;          // queue counter + item arrays
    int32_t* queue = nullptr;
    int32_t* item_group = nullptr;
    int64_t* item_index = nullptr;
    int grid = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // by (full segments, remaining steps) per replay
    std::map<std::pair<int64_t, int64_t>, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
    FusedArgs args{};
    fused_launcher launch = nullptr;
};

extern "C" {

qt_status qt_job_create(qt_context* ctx, const qt_physics* phys, const qt_ttable* tt,
                        const qt_init* init, const qt_batch* batch, int64_t segment_steps,
                        qt_job** out)
{
    if (!ctx || !out) return fail(QT_EINVAL, "null argument");
    if (segment_steps < 1) return fail(QT_EINVAL, "segment_steps must be >= 1");
    std::lock_guard<std::mutex> lk(ctx->mu);
    QT_HIP(hipSetDevice(ctx->device));
    auto* j = new qt_job();
    j->ctx = ctx;
    qt_status st = prepare(ctx, phys, tt, init, batch, &j->hb);
    if (st == QT_OK && batch->form != QT_FORM_FUSED) st = fail(QT_EINVAL, "jobs run the fused form");
    if (st == QT_OK && batch->no_jump_shortcut)
        st = fail(QT_EINVAL, "the no-jump shortcut is not available in segmented jobs");
    if (st == QT_OK) {
        std::vector<HostBatch*> hv{&j->hb};
        st = run_vacuum_phases(ctx, hv, batch->precision, nullptr);
    }
    if (st != QT_OK) {
        delete j;
        return st;
    }
    j->prec = batch->precision;
    j->N = phys->N;
    j->n_traj = batch->n_traj;
    j->seg_steps = segment_steps;
    j->n_steps = j->hb.n_steps;
    auto cleanup = [&](qt_status s) {
        qt_job_destroy(j);
        return s;
    };
    qt_context::Tables t;
    int slots = 0;
    if ((st = pick_launcher(ctx, j->prec, j->N, phys->potential, &j->W, &j->launch, &slots)) != QT_OK)
        return cleanup(st);
    if ((st = ensure_tables(ctx, j->prec, j->N, &t)) != QT_OK) return cleanup(st);
    if ((st = alloc_results(j->n_traj, &j->res)) != QT_OK) return cleanup(st);
    const int64_t n = std::max<int64_t>(j->n_traj, 1);
    if (hipMalloc(reinterpret_cast<void**>(&j->st), n * sizeof(TrajState)) != hipSuccess ||
        hipMalloc(&j->st_psi, (size_t)n * j->N * elem_bytes(j->prec)) != hipSuccess)
        return cleanup(fail(QT_ENOMEM, "no device memory for the job state"));
    QT_HIP(hipMemset(j->st, 0, n * sizeof(TrajState)));
    std::vector<const HostBatch*> hbv{&j->hb};
    std::vector<qt_results> outs{j->res.r};
    if ((st = upload_groups(ctx, hbv, j->prec, outs, false, nullptr, false, &j->dg)) != QT_OK) return cleanup(st);
    j->dg.host[0].st = j->st;
    j->dg.host[0].st_psi = j->st_psi;
    QT_HIP(hipMemcpy(j->dg.groups, j->dg.host.data(), sizeof(GroupDesc), hipMemcpyHostToDevice));
    // items: one group, natural order
    const size_t ib = 256 + al((size_t)n * 4) + (size_t)n * 8;
    QT_HIP(hipMalloc(&j->misc, ib));
    char* m = static_cast<char*>(j->misc);
    j->queue = reinterpret_cast<int32_t*>(m);
    j->item_group = reinterpret_cast<int32_t*>(m + 256);
    j->item_index = reinterpret_cast<int64_t*>(m + 256 + al((size_t)n * 4));
    std::vector<int32_t> ig(n, 0);
    std::vector<int64_t> ii(n);
    for (int64_t i = 0; i < n; ++i) ii[i] = i;
    QT_HIP(hipMemcpy(j->item_group, ig.data(), n * 4, hipMemcpyHostToDevice));
    QT_HIP(hipMemcpy(j->item_index, ii.data(), n * 8, hipMemcpyHostToDevice));
    QT_HIP(hipStreamCreate(&j->stream));
    QT_HIP(hipEventCreateWithFlags(&j->ev_in, hipEventDisableTiming));
    QT_HIP(hipEventCreateWithFlags(&j->ev_out, hipEventDisableTiming));
    j->args.groups = j->dg.groups;
    j->args.item_group = j->item_group;
    j->args.item_index = j->item_index;
    j->args.n_items = (int32_t)j->n_traj;
    j->args.queue = j->queue;
    j->args.tw = t.tw;
    j->args.prew = t.prew;
    j->args.seg_steps = segment_steps;
    j->grid = (int)std::min<int64_t>(std::max<int64_t>(j->n_traj, 1), (int64_t)ctx->n_cu * slots);
    *out = j;
    return QT_OK;
}

qt_status qt_job_advance(qt_job* j, int64_t steps, void* hip_stream)
{
    if (!j || steps < 0) return fail(QT_EINVAL, "bad argument");
    if (steps == 0 || j->n_traj == 0) return QT_OK;
    std::lock_guard<std::mutex> lk(j->ctx->mu);
    QT_HIP(hipSetDevice(j->ctx->device));
    // `steps` steps exactly: full segments, then one launch of the remainder
    const int64_t full = steps / j->seg_steps, rem = steps % j->seg_steps;
    const int64_t launches = full + (rem > 0 ? 1 : 0);
    const auto key = std::make_pair(full, rem);
    auto it = j->graphs.find(key);
    if (it == j->graphs.end()) {
        // capture the launches once, replay afterwards
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        QT_HIP(hipStreamBeginCapture(j->stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        FusedArgs last = j->args;
        last.seg_steps = rem;
        for (int64_t k = 0; k < launches && e == hipSuccess; ++k) {
            e = launch_queue_reset(j->queue, j->stream);
            if (e == hipSuccess) e = j->launch(k < full ? j->args : last, j->grid, j->stream);
        }
        hipError_t e2 = hipStreamEndCapture(j->stream, &g);
        if (e != hipSuccess) return fail(QT_EDEVICE, "capture failed: %s", hipGetErrorString(e));
        if (e2 != hipSuccess) return fail(QT_EDEVICE, "end capture failed: %s", hipGetErrorString(e2));
        QT_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
        it = j->graphs.emplace(key, std::make_pair(g, ge)).first;
    }
    hipStream_t us = static_cast<hipStream_t>(hip_stream);
    QT_HIP(hipEventRecord(j->ev_in, us));
    QT_HIP(hipStreamWaitEvent(j->stream, j->ev_in, 0));
    QT_HIP(hipEventRecord(j->ctx->ev0, j->stream));
    QT_HIP(hipGraphLaunch(it->second.second, j->stream));
    QT_HIP(hipEventRecord(j->ctx->ev1, j->stream));
    QT_HIP(hipEventRecord(j->ev_out, j->stream));
    QT_HIP(hipStreamWaitEvent(us, j->ev_out, 0));
    j->ctx->timed = true;
    j->ctx->last_launches = 2 * launches;
    if (trace_on()) {
        QT_HIP(hipEventSynchronize(j->ctx->ev1));
        float ms = 0.f;
        QT_HIP(hipEventElapsedTime(&ms, j->ctx->ev0, j->ctx->ev1));
        trace_line("{\"event\": \"segment\", \"N\": %d, \"precision\": %d, \"trajectories\": %lld, "
                   "\"steps\": %lld, \"launches\": %lld, \"kernel_ms\": %.3f}",
                   j->N, j->prec, (long long)j->n_traj, (long long)steps, (long long)launches, ms);
    }
    return QT_OK;
}

qt_status qt_job_done(qt_job* j, int32_t* done)
{
    if (!j || !done) return fail(QT_EINVAL, "null argument");
    QT_HIP(hipSetDevice(j->ctx->device));
    QT_HIP(hipStreamSynchronize(j->stream));
    std::vector<TrajState> h((size_t)j->n_traj);
    if (j->n_traj) QT_HIP(hipMemcpy(h.data(), j->st, h.size() * sizeof(TrajState), hipMemcpyDeviceToHost));
    int32_t d = 1;
    for (const TrajState& s : h)
        if (!s.done) { d = 0; break; }
    *done = d;
    return QT_OK;
}

qt_status qt_job_state_bytes(qt_job* j, size_t* bytes)
{
    if (!j || !bytes) return fail(QT_EINVAL, "null argument");
    const int64_t n = std::max<int64_t>(j->n_traj, 1);
    *bytes = n * sizeof(TrajState) + (size_t)n * j->N * elem_bytes(j->prec) + j->res.bytes;
    return QT_OK;
}

// state = [TrajState x n | psi | results block]
static qt_status job_copy(qt_job* j, void* dst, const void* src, bool save, void* hip_stream)
{
    QT_HIP(hipSetDevice(j->ctx->device));
    hipStream_t us = static_cast<hipStream_t>(hip_stream);
    QT_HIP(hipEventRecord(j->ev_in, j->stream));
    QT_HIP(hipStreamWaitEvent(us, j->ev_in, 0));
    const int64_t n = std::max<int64_t>(j->n_traj, 1);
    const size_t a = n * sizeof(TrajState), b = (size_t)n * j->N * elem_bytes(j->prec);
    if (save) {
        char* d = static_cast<char*>(dst);
        QT_HIP(hipMemcpyAsync(d, j->st, a, hipMemcpyDefault, us));
        QT_HIP(hipMemcpyAsync(d + a, j->st_psi, b, hipMemcpyDefault, us));
        QT_HIP(hipMemcpyAsync(d + a + b, j->res.mem, j->res.bytes, hipMemcpyDefault, us));
    } else {
        const char* s = static_cast<const char*>(src);
        QT_HIP(hipMemcpyAsync(j->st, s, a, hipMemcpyDefault, us));
        QT_HIP(hipMemcpyAsync(j->st_psi, s + a, b, hipMemcpyDefault, us));
        QT_HIP(hipMemcpyAsync(j->res.mem, s + a + b, j->res.bytes, hipMemcpyDefault, us));
    }
    QT_HIP(hipEventRecord(j->ev_out, us));
    QT_HIP(hipStreamWaitEvent(j->stream, j->ev_out, 0));
    return QT_OK;
}

qt_status qt_job_save(qt_job* j, void* dst, void* hip_stream)
{
    if (!j || !dst) return fail(QT_EINVAL, "null argument");
    return job_copy(j, dst, nullptr, true, hip_stream);
}

qt_status qt_job_load(qt_job* j, const void* src, void* hip_stream)
{
    if (!j || !src) return fail(QT_EINVAL, "null argument");
    return job_copy(j, nullptr, src, false, hip_stream);
}

qt_status qt_job_results(qt_job* j, const qt_results* dev_out, void* hip_stream)
{
    if (!j || !dev_out) return fail(QT_EINVAL, "null argument");
    if (dev_out->jump_log) return fail(QT_EINVAL, "a job keeps no jump log");
    QT_HIP(hipSetDevice(j->ctx->device));
    hipStream_t us = static_cast<hipStream_t>(hip_stream);
    QT_HIP(hipEventRecord(j->ev_in, j->stream));
    QT_HIP(hipStreamWaitEvent(us, j->ev_in, 0));
    qt_status st = copy_results(j->res.r, *dev_out, j->n_traj, hipMemcpyDeviceToDevice, us);
    if (st != QT_OK) return st;
    if (dev_out->psi) QT_HIP(launch_widen(j->st_psi, j->prec, dev_out->psi, j->n_traj * j->N, us));
    return QT_OK;
}

qt_status qt_job_destroy(qt_job* j)
{
    if (!j) return QT_OK;
    hipSetDevice(j->ctx->device);
    if (j->stream) hipStreamSynchronize(j->stream);
    for (auto& kv : j->graphs) {
        hipGraphExecDestroy(kv.second.second);
        hipGraphDestroy(kv.second.first);
    }
    if (j->stream) hipStreamDestroy(j->stream);
    if (j->ev_in) hipEventDestroy(j->ev_in);
    if (j->ev_out) hipEventDestroy(j->ev_out);
    hipFree(j->misc);
    hipFree(j->st);
    hipFree(j->st_psi);
    hipFree(j->res.mem);
    hipFree(j->dg.mem);
    delete j;
    return QT_OK;
}

}  // extern "C"
