// qt_host.hpp -- host-side runtime shared by the C ABI entry points.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "qt_internal.h"

struct qt_context {
    int device = 0;
    int n_cu = 0;
    std::mutex mu;
    struct Tables { void* tw = nullptr; void* prew = nullptr; };
    std::map<std::pair<int, int>, Tables> tables;          // (precision, N)
    struct Variant { int W = 0; int slots_per_cu = 0; bool tuned = false; };
    std::map<std::pair<int, int>, Variant> plans;          // (precision, N)
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool timed = false;
    int64_t last_launches = 0;
    std::vector<hipStream_t> aux;                          // fork/join streams
    std::vector<hipEvent_t> join;                          // their join events
    hipEvent_t fork = nullptr;                             // the fork point
    // static phase tables exp(-i dt/2 V_static) per (l, colour), keyed by
    // (precision, N, L, mass, alpha_s, dt)
    std::map<std::vector<double>, void*> phase;
    // (phi, phi') table of the KSU potential's imaginary part, per precision
    std::map<int, void*> ksu_phi;
    // vacuum eigenstates (energies[6] then basis[6 N]) keyed by (N, L, mass,
    // alpha_s, deriv_type, potential); their own lock: requests are
    // prepared outside `mu` by the server
    std::mutex eig_mu;
    struct Eigen {
        double energies[6];
        std::shared_ptr<const std::vector<double>> basis;   // 6 N
    };
    std::map<std::vector<double>, Eigen> eigen;
    // this device's copy of the library's static no-allocation buffer
    // (qt_run_noalloc), looked up when the context is created
    void* noalloc_buf = nullptr;
};

namespace qt {

qt_status fail(qt_status s, const char* fmt, ...);

// QTRAJ_TRACE (environment): when it names a file (or "stderr"), runs, job
// segments and server rounds each append one JSON line there, after their
// device work has finished (tracing synchronises the stream it traces).
bool trace_on();
void trace_line(const char* fmt, ...);

// Set while the calling thread runs qt_run_noalloc: a context table, basis or
// plan that would have to be built (device allocation) is an error instead.
extern thread_local bool g_no_alloc;
// The device address of the static no-allocation buffer on `device` (looked
// up once per device, with the device current) and its size.
qt_status noalloc_buffer(int device, void** ptr, size_t* bytes);
#define QT_HIP(x)                                                                         \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess) return ::qt::fail(QT_EDEVICE, "%s failed: %s", #x,          \
                                                hipGetErrorString(e_));                   \
    } while (0)

int elem_bytes(int prec);     // bytes of one complex value of the precision
double kinetic_energy(const qt_physics* p, int k);   // of sine mode k
// vacuum eigenstates 1S, 2S, 1P, 3S, 2P, 1D (qt_eigen.cpp): energies [6],
// basis [6 N] (host memory); computed once per context and parameters
qt_status eigen_states(qt_context* ctx, const qt_physics* p, qt_context::Eigen* out);

// Initial state (2N, normalised) and its overlaps with the six Coulomb
// states.
struct InitTable {
    std::vector<double> psi;
    double overlap[6] = {0, 0, 0, 0, 0, 0};
};

// Host copy of one batch's setup (everything the device needs, in FP64).
// The N-sized tables are shared between all batches with the same
// parameters (see prepare), and uploaded once per launch.
struct HostBatch {
    qt_physics phys;
    qt_batch batch;
    int init_l = 0, init_color = 0;
    int64_t n_steps = 0;
    std::vector<double> tau, T;
    double tau_start = 0, T_final = 0;
    std::shared_ptr<const std::vector<double>> kin;     // 2N: (2/N) exp(-i E_k dt)
    std::shared_ptr<const std::vector<double>> basis;   // 6N
    std::shared_ptr<const InitTable> init;
    int64_t vacuum_steps = 0;       // in-vacuum steps before the medium (once)
    qt_results zeroth{};            // device results of the zeroth trajectory
    int32_t* zdone = nullptr;       // its completion flag (device)
};

qt_status validate(const qt_physics* p, const qt_ttable* tt, const qt_init* in,
                   const qt_batch* b);
qt_status prepare(qt_context* ctx, const qt_physics* p, const qt_ttable* tt, const qt_init* in,
                  const qt_batch* b, HostBatch* out);
int64_t count_steps(const qt_physics& p, const qt_ttable& tt);
double host_temperature(const double* tau, const double* T, int n, double t);

qt_status ensure_tables(qt_context* ctx, int prec, int N, qt_context::Tables* out);
qt_status choose_variant(qt_context* ctx, int prec, int N, qt_context::Variant* out);
// The fused kernel for (precision, N, potential): block size, launcher and
// resident workgroups per CU (the tuned variant for the Munich potential).
qt_status pick_launcher(qt_context* ctx, int prec, int N, int potential, int* W,
                        fused_launcher* launch, int* slots_per_cu);

// Device image of a set of groups: one allocation holding group descriptors
// and every table they point to.  `kin` is converted to the precision.
struct DeviceGroups {
    void* mem = nullptr;
    size_t bytes = 0;
    GroupDesc* groups = nullptr;     // device
    std::vector<GroupDesc> host;     // host copy
};
// `into` (optional): device memory of `into_cap` bytes to build the image in
// instead of an allocation (QT_EINVAL when it does not fit).
qt_status upload_groups(qt_context* ctx, const std::vector<const HostBatch*>& hb, int prec,
                        const std::vector<qt_results>& outs, bool with_Tn,
                        hipStream_t s, bool async_alloc, DeviceGroups* out,
                        void* into = nullptr, size_t into_cap = 0);
qt_status ensure_phase(qt_context* ctx, const HostBatch& hb, int prec, const void** out);
qt_status ensure_ksu_table(qt_context* ctx, int prec, const void** out);

// Device buffers for the per-trajectory results (no wave functions).
struct ResultBuffers {
    void* mem = nullptr;
    size_t bytes = 0;
    qt_results r{};
};
qt_status alloc_results(int64_t n, ResultBuffers* rb);
size_t result_bytes(int64_t n);
qt_status copy_results(const qt_results& src, const qt_results& dst, int64_t n, hipMemcpyKind kind,
                       hipStream_t s);
qt_status run_fused_groups(qt_context* ctx, const std::vector<const HostBatch*>& hb,
                           const std::vector<qt_results>& outs, int prec, hipStream_t s);

// Runs the in-vacuum phase (T = 0, no jumps, vacuum_steps steps) of every
// batch that has one, all in one launch, and makes its result the batch's
// initial state.  Synchronises `s`.
qt_status run_vacuum_phases(qt_context* ctx, const std::vector<HostBatch*>& hb, int prec,
                            hipStream_t s);
// For every batch that asks for the no-jump shortcut: a zeroth (no-jump)
// trajectory group is appended to v/outs (stored in *zb) for the same launch,
// and the batch is pointed at its results and completion flag (device
// memory in *mem, which the caller frees stream-ordered after the launch).
qt_status add_zeroth_groups(const std::vector<HostBatch*>& hb, std::vector<HostBatch>* zb,
                            std::vector<const HostBatch*>* v, std::vector<qt_results>* outs,
                            hipStream_t s, void** mem);

// One persistent launch of the fused kernel (one class of items).
struct ClassLaunch {
    fused_launcher launch = nullptr;
    FusedArgs args{};
    int grid = 0;
};
// Launches the classes concurrently: the first on `s`, the others on fork
// streams of default priority (created into `streams`/`joins` as needed,
// owned by the caller, which must not use them from two threads at once),
// each after `fork` recorded on `s` and joined back into `s`.  Each launch
// is preceded by its queue reset on its own stream.
qt_status launch_classes(const std::vector<ClassLaunch>& v, hipStream_t s, hipEvent_t* fork,
                         std::vector<hipStream_t>* streams, std::vector<hipEvent_t>* joins);

// LPT order of (group, index) items: longest remaining work first.
void build_items(const std::vector<const HostBatch*>& hb, std::vector<int32_t>* ig,
                 std::vector<int64_t>* ii);

}  // namespace qt
