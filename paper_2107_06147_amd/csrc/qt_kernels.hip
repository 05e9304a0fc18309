// qt_kernels.hip -- HIP kernels (gfx950) of the quantum-trajectory solver.
//
// FUSED form: one persistent kernel.  Each workgroup of W lanes pops a
// trajectory from a device queue, loads its wave function into registers
// (mirror layout, see qt_device.hpp) and runs the whole time loop on chip:
//   K-multiply -> DST-I -> kinetic multiply -> DST-I -> K-multiply -> norm,
// then the jump decision (paper: Sec. "Algorithm for deterministic evolution
// between quantum jumps", the five sub-steps; Sec. "The waiting time
// approach" and "Summary of QTraj execution", step 4, for the jump).  HBM is
// touched only to load the initial state, at segment checkpoints, and for
// the results.  When the trajectory retires the workgroup pops the next one.
//
// PLAIN form (FP64): one kernel per sub-step per time step, the wave
// function in HBM between kernels.  It is the unfused baseline.
//
// Precision R = float is the FP32-bulk form: wave function, transforms and
// multiplies in FP32; the norm is accumulated in FP64 and compared with the
// FP64 threshold; the static potential phase and all per-step scalars are
// computed in FP64 and rounded once.
#include "qt_fused.hpp"

namespace qt {

__global__ void queue_reset_kernel(int32_t* q) { *q = 0; }

__global__ void zero_i32_kernel(int32_t* p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

hipError_t launch_zero_i32(int32_t* p, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    zero_i32_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

template <class R>
__global__ void widen_kernel(const cx<R>* src, double* dst, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    dst[2 * i] = (double)src[i].re;
    dst[2 * i + 1] = (double)src[i].im;
}

hipError_t launch_widen(const void* src, int prec, double* dst, int64_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    const dim3 grid((unsigned)((count + 255) / 256));
    if (prec == QT_FP32_BULK)
        hipLaunchKernelGGL(widen_kernel<float>, grid, dim3(256), 0, s,
                           static_cast<const cx<float>*>(src), dst, count);
    else
        hipLaunchKernelGGL(widen_kernel<double>, grid, dim3(256), 0, s,
                           static_cast<const cx<double>*>(src), dst, count);
    return hipGetLastError();
}

hipError_t launch_queue_reset(int32_t* q, hipStream_t s)
{
    hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(1), 0, s, q);
    return hipGetLastError();
}

#define QT_F32(N, W) {QT_FP32_BULK, N, W, launch_fused<float, N, W, 0>, occupancy_fused<float, N, W, 0>}
#define QT_F64(N, W) {QT_FP64, N, W, launch_fused<double, N, W, 0>, occupancy_fused<double, N, W, 0>}

static const FusedEntry kFused[] = {
    // FP32-bulk: 8..16 complex values per lane (4 only at N = 256, whose
    // transform then runs in FP64)
    QT_F32(256, 64),   QT_F32(512, 64),   QT_F32(1024, 64),  QT_F32(1024, 128),
    QT_F32(2048, 128), QT_F32(2048, 256), QT_F32(4096, 256), QT_F32(4096, 512),
    QT_F32(8192, 512), QT_F32(8192, 1024),
    // FP64: 4..8 complex values per lane
    QT_F64(256, 64),   QT_F64(512, 64),   QT_F64(512, 128),  QT_F64(1024, 128),
    QT_F64(1024, 256), QT_F64(2048, 256), QT_F64(2048, 512), QT_F64(4096, 512),
    QT_F64(4096, 1024), QT_F64(8192, 1024),
};

int fused_variants(int prec, int N, int* W_out, int max_out)
{
    int n = 0;
    for (const auto& e : kFused)
        if (e.prec == prec && e.N == N && n < max_out) W_out[n++] = e.W;
    return n;
}

fused_launcher fused_get(int prec, int N, int W)
{
    for (const auto& e : kFused)
        if (e.prec == prec && e.N == N && e.W == W) return e.launch;
    return nullptr;
}

int fused_occupancy(int prec, int N, int W)
{
    for (const auto& e : kFused)
        if (e.prec == prec && e.N == N && e.W == W) return e.occ();
    return 0;
}

// ------------------------------------------------------------ PLAIN -------
// One thread per grid point or one workgroup per trajectory; psi in HBM in
// natural order (2N doubles per trajectory).

__global__ void plain_space_kernel(const GroupDesc* gp, double* psi, const TrajState* st,
                                   int64_t n_traj, int N, int64_t n)
{
    const GroupDesc& g = *gp;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tr = gid / N;
    const int m = (int)(gid % N);
    if (tr >= n_traj || m == 0) return;
    const TrajState& s = st[tr];
    if (s.done) return;
    // the half-step factor exp(-i V_eff dt/2) at T_n from the full potential
    const double T = g.Tn[n];
    const double T3 = T * T * T;
    const double r = (double)m * g.dr;
    const double cent = (double)s.l * (double)(s.l + 1) / (g.mass * r * r);
    double VR, VI;
    if (g.potential == QT_POTENTIAL_KSU) {
        double md, cI;
        ksu_medium(T, g.md_factor, &md, &cI);
        const double rsb = 1.25 / 0.1973269804;
        const HalfStepKSU<double> h{static_cast<const cx<double>*>(g.ksu_phi), g.dr, 0.0, md, cI,
                                    0.0, -kKsuA / rsb + kKsuSigma * rsb};
        const double x = md * r;
        const double q = x > 1e-4 ? -expm1(-x) / x : 1.0 - x * (0.5 - x / 6.0);
        const double e = exp(-x);
        const double kms = -(kKsuA / r) * (1.0 + x) * e + 2.0 * kKsuSigma * r * q - kKsuSigma * r * e;
        VR = (kms <= h.vsb ? kms : h.vsb) + cent;
        VI = -cI * h.phi(x);
    } else if (s.c == QT_SINGLET) {
        VR = -g.alpha / r + 0.5 * g.gamma_hat * T3 * r * r + cent;
        VI = -0.5 * kappa_hat_at(g.kappa_hat, T) * T3 * r * r;
    } else {
        VR = g.alpha / (8.0 * r) + (7.0 / 32.0) * g.gamma_hat * T3 * r * r + cent;
        VI = -(7.0 / 32.0) * kappa_hat_at(g.kappa_hat, T) * T3 * r * r;
    }
    const double mag = exp(0.5 * g.dt * VI);
    double sn, cs;
    sincos(-0.5 * g.dt * VR, &sn, &cs);
    const double kr = mag * cs, ki = mag * sn;
    double* u = psi + (size_t)tr * 2 * N + 2 * m;
    const double ur = u[0], ui = u[1];
    u[0] = ur * kr - ui * ki;
    u[1] = ur * ki + ui * kr;
}

__global__ void plain_kinetic_kernel(const GroupDesc* gp, double* psi, const TrajState* st,
                                     int64_t n_traj, int N)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tr = gid / N;
    const int m = (int)(gid % N);
    if (tr >= n_traj) return;
    if (st[tr].done) return;
    const double* kin = static_cast<const double*>(gp->kin);
    double* u = psi + (size_t)tr * 2 * N + 2 * m;
    const double ur = u[0], ui = u[1];
    const double kr = kin[2 * m], ki = kin[2 * m + 1];
    u[0] = ur * kr - ui * ki;
    u[1] = ur * ki + ui * kr;
}

template <int N, int W>
__global__ __launch_bounds__(W) void plain_dst_kernel(double* psi, const TrajState* st,
                                                      const void* twv, const void* prewv)
{
    using PL = Plan<N, W>;
    constexpr int R1 = PL::R1, T = PL::T;
    __shared__ cx<double> buf[padded_len<N>()];
    __shared__ cx<double> wsum[W / 64];
    const int64_t tr = blockIdx.x;
    if (st[tr].done) return;
    const Lanes<N, W> ln(threadIdx.x);
    const cx<double>* prew = static_cast<const cx<double>*>(prewv);
    cx<double> a[R1], b[R1];
    cx<double>* u = reinterpret_cast<cx<double>*>(psi) + (size_t)tr * N;
    sfor<0, R1>([&](auto Rr) QT_INL {
        a[Rr] = u[ln.ja + Rr * T];
        b[Rr] = u[ln.jb + Rr * T];
    });
    cx<double> pw[Plan<N, W>::R1];
    load_prew<double, N, W>(pw, prew, ln);
    dst1<double, N, W, false>(a, b, pw, prew, ln, buf, wsum, static_cast<const cx<double>*>(twv), nullptr);
    sfor<0, R1>([&](auto Rr) QT_INL {
        u[ln.ja + Rr * T] = a[Rr];
        u[ln.jb + Rr * T] = b[Rr];
    });
}

template <int W>
__global__ __launch_bounds__(W) void plain_init_kernel(const GroupDesc* gp, double* psi,
                                                       TrajState* st, int N)
{
    __shared__ double red[W / 64];
    const GroupDesc& g = *gp;
    const int64_t tr = blockIdx.x;
    double acc = 0.0;
    for (int m = threadIdx.x; m < N; m += W) {
        const double ur = g.init_psi[2 * m], ui = g.init_psi[2 * m + 1];
        psi[(size_t)tr * 2 * N + 2 * m] = ur;
        psi[(size_t)tr * 2 * N + 2 * m + 1] = ui;
        acc += ur * ur + ui * ui;
    }
    const double nrm = g.dr * block_sum<W>(acc, red);
    if (threadIdx.x == 0) {
        const uint64_t stride = g.traj_id_stride ? g.traj_id_stride : 1u;
        const U4 e0 = event_block(g.seed, g.traj_id0 + (uint64_t)tr * stride, 0);
        TrajState s;
        s.step = 0; s.l = g.init_l; s.c = g.init_color; s.n_jumps = 0;
        s.r = uniform01(e0.w[2]); s.first_r = s.r; s.min_gap = __builtin_huge_val();
        s.norm = nrm; s.started = 1; s.pad0 = 0; s.pad1 = 0; s.scl = 1.0; s.pad2 = 0.0;
        s.status = (g.do_jumps && s.r > g.r_max) ? QT_TRAJ_RMAX : QT_TRAJ_OK;
        s.done = (s.status != QT_TRAJ_OK || g.n_steps == 0) ? 1 : 0;
        st[tr] = s;
    }
}

template <int W>
__global__ __launch_bounds__(W) void plain_norm_jump_kernel(const GroupDesc* gp, double* psi,
                                                            TrajState* st, int N, int64_t n)
{
    __shared__ double red[W / 64];
    const GroupDesc& g = *gp;
    const int64_t tr = blockIdx.x;
    TrajState s = st[tr];
    if (s.done) return;
    double* u = psi + (size_t)tr * 2 * N;
    auto norm_now = [&]() QT_INL {
        double acc = 0.0;
        for (int m = threadIdx.x; m < N; m += W) acc += u[2 * m] * u[2 * m] + u[2 * m + 1] * u[2 * m + 1];
        return g.dr * block_sum<W>(acc, red);
    };
    s.norm = norm_now();
    s.step = n + 1;
    if (g.do_jumps) {
        const double gap = fabs(s.norm - s.r);
        if (gap < s.min_gap) s.min_gap = gap;
        if (s.norm <= s.r) {
            if (g.max_jumps >= 0 && s.n_jumps >= g.max_jumps) {
                s.status = QT_TRAJ_MAXJUMPS;
            } else {
                const uint64_t stride = g.traj_id_stride ? g.traj_id_stride : 1u;
                const U4 e = event_block(g.seed, g.traj_id0 + (uint64_t)tr * stride,
                                         (int64_t)s.n_jumps + 1);
                const double ul = uniform01(e.w[0]), uc = uniform01(e.w[1]);
                s.l = (ul < (double)s.l / (double)(2 * s.l + 1)) ? s.l - 1 : s.l + 1;
                s.c = (s.c == QT_OCTET) ? (uc < 2.0 / 7.0 ? QT_SINGLET : QT_OCTET) : QT_OCTET;
                log_jump(g.out, tr, s.n_jumps, n, s.l, s.c);
                double acc = 0.0;
                for (int m = threadIdx.x; m < N; m += W) {
                    const double rm = (double)m * g.dr;
                    u[2 * m] *= rm;
                    u[2 * m + 1] *= rm;
                    acc += u[2 * m] * u[2 * m] + u[2 * m + 1] * u[2 * m + 1];
                }
                const double f = 1.0 / sqrt(g.dr * block_sum<W>(acc, red));
                for (int m = threadIdx.x; m < N; m += W) {
                    u[2 * m] *= f;
                    u[2 * m + 1] *= f;
                }
                __syncthreads();
                s.norm = norm_now();
                s.r = uniform01(e.w[2]);
                s.n_jumps += 1;
            }
        }
    }
    if (s.status != QT_TRAJ_OK || s.step >= g.n_steps) s.done = 1;
    __syncthreads();
    if (threadIdx.x == 0) st[tr] = s;
}

template <int W>
__global__ __launch_bounds__(W) void plain_finalize_kernel(const GroupDesc* gp, const double* psi,
                                                           const TrajState* st, int N)
{
    __shared__ double red[14 * (W / 64)];
    const GroupDesc& g = *gp;
    const int64_t tr = blockIdx.x;
    const TrajState s = st[tr];
    const double* u = psi + (size_t)tr * 2 * N;
    double x[14];
#pragma unroll
    for (int i = 0; i < 14; ++i) x[i] = 0.0;
    for (int m = threadIdx.x; m < N; m += W) {
        const double ur = u[2 * m], ui = u[2 * m + 1];
        const double w2 = ur * ur + ui * ui;
        x[12] += w2;
        x[13] += (double)m * g.dr * w2;
#pragma unroll
        for (int bb = 0; bb < 6; ++bb) {
            const double ph = g.basis[bb * N + m];
            x[2 * bb] += ph * ur;
            x[2 * bb + 1] += ph * ui;
        }
    }
    block_sum_vec<W, 14>(x, red);
    const qt_results& o = g.out;
    if (threadIdx.x == 0) {
        constexpr int basis_l[6] = {0, 0, 1, 0, 1, 2};
        const double nrm = x[12];
#pragma unroll
        for (int bb = 0; bb < 6; ++bb) {
            double ov = 0.0, sv = 0.0;
            if (s.status == QT_TRAJ_OK && s.c == QT_SINGLET && s.l == basis_l[bb] && nrm > 0.0) {
                const double dr_ = g.dr * x[2 * bb], di_ = g.dr * x[2 * bb + 1];
                ov = (dr_ * dr_ + di_ * di_) / (g.dr * nrm);
                // (an initial population below 1e-12 is rounding: no ratio)
                sv = g.init_overlap[bb] > 1e-12 ? ov / g.init_overlap[bb] : ov;
            }
            if (o.overlap) o.overlap[6 * tr + bb] = ov;
            if (o.survival) o.survival[6 * tr + bb] = sv;
        }
        if (o.norm) o.norm[tr] = s.norm;
        if (o.first_r) o.first_r[tr] = s.first_r;
        if (o.mean_r) o.mean_r[tr] = nrm > 0.0 ? x[13] / nrm : 0.0;
        if (o.l) o.l[tr] = s.l;
        if (o.color) o.color[tr] = s.c;
        if (o.n_jumps) o.n_jumps[tr] = s.n_jumps;
        if (o.status) o.status[tr] = s.status;
        if (o.steps_done) o.steps_done[tr] = s.step;
        if (o.min_gap) o.min_gap[tr] = s.min_gap;
    }
    if (o.psi) {
        for (int m = threadIdx.x; m < N; m += W) {
            o.psi[(size_t)tr * 2 * N + 2 * m] = u[2 * m];
            o.psi[(size_t)tr * 2 * N + 2 * m + 1] = u[2 * m + 1];
        }
    }
}

constexpr int kPlainW = 256;

hipError_t plain_init(const PlainArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(plain_init_kernel<kPlainW>, dim3((unsigned)a.n_traj), dim3(kPlainW), 0, s,
                       a.g, a.psi, a.st, a.N);
    return hipGetLastError();
}

static dim3 elementwise_grid(const PlainArgs& a)
{
    return dim3((unsigned)((a.n_traj * a.N + 255) / 256));
}

hipError_t plain_space(const PlainArgs& a, int64_t n, hipStream_t s)
{
    dim3 grid = elementwise_grid(a);
    hipLaunchKernelGGL(plain_space_kernel, grid, dim3(256), 0, s, a.g, a.psi, a.st, a.n_traj,
                       a.N, n);
    return hipGetLastError();
}

hipError_t plain_kinetic(const PlainArgs& a, hipStream_t s)
{
    dim3 grid = elementwise_grid(a);
    hipLaunchKernelGGL(plain_kinetic_kernel, grid, dim3(256), 0, s, a.g, a.psi, a.st, a.n_traj,
                       a.N);
    return hipGetLastError();
}

template <int N, int W>
static hipError_t plain_dst_n(const PlainArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL((plain_dst_kernel<N, W>), dim3((unsigned)a.n_traj), dim3(W), 0, s, a.psi,
                       a.st, a.tw, a.prew);
    return hipGetLastError();
}

bool plain_supported(int N)
{
    return N == 256 || N == 512 || N == 1024 || N == 2048 || N == 4096 || N == 8192;
}

hipError_t plain_dst(const PlainArgs& a, hipStream_t s)
{
    switch (a.N) {
    case 256: return plain_dst_n<256, 64>(a, s);
    case 512: return plain_dst_n<512, 64>(a, s);
    case 1024: return plain_dst_n<1024, 128>(a, s);
    case 2048: return plain_dst_n<2048, 256>(a, s);
    case 4096: return plain_dst_n<4096, 256>(a, s);
    case 8192: return plain_dst_n<8192, 512>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t plain_norm_jump(const PlainArgs& a, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(plain_norm_jump_kernel<kPlainW>, dim3((unsigned)a.n_traj), dim3(kPlainW), 0,
                       s, a.g, a.psi, a.st, a.N, n);
    return hipGetLastError();
}

hipError_t plain_finalize(const PlainArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(plain_finalize_kernel<kPlainW>, dim3((unsigned)a.n_traj), dim3(kPlainW), 0,
                       s, a.g, a.psi, a.st, a.N);
    return hipGetLastError();
}

}  // namespace qt
