// qt_noalloc.hip -- qt_run without device allocation (qt_run_noalloc).
//
// The per-call device data of a fused run (queue counter, work items, group
// descriptor and its tables) goes into one static device buffer of the
// library instead of a hipMalloc'ed one.  Each device holds its own copy of
// the buffer for the life of the process; every call on a device shares it,
// so calls that overlap on one device race (the caller serialises them, for
// example on one stream).  The buffer keeps the last call's contents: the
// queue counter is cleared by a fill kernel at every launch, and every other
// byte that a launch reads is written by the same call first.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <vector>

#include "qt_host.hpp"

// The buffer itself.  In host code its name stands for a host-side shadow,
// not a device address: it is only ever used through the address that
// hipGetSymbolAddress returns for the current device (noalloc_buffer).
static __device__ __align__(256) char scratch[QT_NOALLOC_BUFFER_BYTES];

namespace qt {

qt_status noalloc_buffer(int device, void** ptr, size_t* bytes)
{
    static std::mutex mu;
    static std::map<int, void*> addr;
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(device);
    if (it == addr.end()) {
        int cur = 0;
        QT_HIP(hipGetDevice(&cur));
        QT_HIP(hipSetDevice(device));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        (void)hipSetDevice(cur);
        if (e != hipSuccess || p == nullptr)
            return fail(QT_EDEVICE, "hipGetSymbolAddress of the static buffer failed on device %d: %s",
                        device, hipGetErrorString(e));
        it = addr.emplace(device, p).first;
    }
    *ptr = it->second;
    *bytes = QT_NOALLOC_BUFFER_BYTES;
    return QT_OK;
}

}  // namespace qt

using namespace qt;

namespace {

// g_no_alloc for the duration of one call
struct NoAllocScope {
    NoAllocScope() { g_no_alloc = true; }
    ~NoAllocScope() { g_no_alloc = false; }
};

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

extern "C" qt_status qt_run_noalloc(qt_context* ctx, const qt_physics* phys, const qt_ttable* tt,
                                    const qt_init* init, const qt_batch* batch,
                                    const qt_results* dev_out, void* hip_stream)
{
    if (!ctx || !phys || !tt || !init || !batch || !dev_out) return fail(QT_EINVAL, "null argument");
    if (dev_out->jump_log_cap < 0) return fail(QT_EINVAL, "jump_log_cap < 0");
    if (batch->form != QT_FORM_FUSED) return fail(QT_EINVAL, "qt_run_noalloc runs the fused form");
    if (batch->no_jump_shortcut)
        return fail(QT_EINVAL, "the no-jump shortcut is not available in qt_run_noalloc");
    if (tt->vacuum_steps > 0) return fail(QT_EINVAL, "a vacuum phase is not available in qt_run_noalloc");
    std::lock_guard<std::mutex> lk(ctx->mu);
    QT_HIP(hipSetDevice(ctx->device));
    if (!ctx->noalloc_buf) return fail(QT_EDEVICE, "no static buffer on device %d", ctx->device);
    NoAllocScope scope;
    HostBatch hb;
    qt_status st = prepare(ctx, phys, tt, init, batch, &hb);
    if (st != QT_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    // [queue counter | item groups (n int32) | item indices (n int64) | group image]
    const int64_t n = batch->n_traj;
    const size_t cap = QT_NOALLOC_BUFFER_BYTES;
    const size_t o_ig = 256, o_ii = o_ig + up256((size_t)n * 4), o_img = o_ii + up256((size_t)n * 8);
    if (o_img > cap)
        return fail(QT_EINVAL, "%lld trajectories need %zu bytes of work items, more than the %zu-byte "
                    "static buffer", (long long)n, o_img, cap);
    char* base = static_cast<char*>(ctx->noalloc_buf);
    std::vector<const HostBatch*> v{&hb};
    std::vector<qt_results> outs{*dev_out};
    DeviceGroups dg;
    if ((st = upload_groups(ctx, v, batch->precision, outs, false, s, false, &dg, base + o_img,
                            cap - o_img)) != QT_OK)
        return st;
    int W = 0, slots = 0;
    fused_launcher launch = nullptr;
    if ((st = pick_launcher(ctx, batch->precision, phys->N, phys->potential, &W, &launch, &slots)) != QT_OK)
        return st;
    qt_context::Tables t;
    if ((st = ensure_tables(ctx, batch->precision, phys->N, &t)) != QT_OK) return st;
    QT_HIP(hipEventRecord(ctx->ev0, s));
    if (n > 0) {
        // one batch: its trajectories in order (equal lengths: LPT is the order itself)
        std::vector<int32_t> ig((size_t)n, 0);
        std::vector<int64_t> ii((size_t)n);
        for (int64_t i = 0; i < n; ++i) ii[(size_t)i] = i;
        QT_HIP(hipMemcpyAsync(base + o_ig, ig.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
        QT_HIP(hipMemcpyAsync(base + o_ii, ii.data(), (size_t)n * 8, hipMemcpyHostToDevice, s));
        // the copies read pageable memory: wait for them before it goes away
        QT_HIP(hipStreamSynchronize(s));
        FusedArgs a;
        a.groups = dg.groups;
        a.item_group = reinterpret_cast<const int32_t*>(base + o_ig);
        a.item_index = reinterpret_cast<const int64_t*>(base + o_ii);
        a.n_items = (int32_t)n;
        a.queue = reinterpret_cast<int32_t*>(base);
        a.tw = t.tw;
        a.prew = t.prew;
        a.seg_steps = 0;
        const int grid = (int)std::min<int64_t>(n, (int64_t)ctx->n_cu * slots);
        QT_HIP(launch_queue_reset(a.queue, s));
        QT_HIP(launch(a, grid, s));
    }
    QT_HIP(hipEventRecord(ctx->ev1, s));
    ctx->timed = true;
    ctx->last_launches = n > 0 ? 2 : 0;
    return QT_OK;
}
