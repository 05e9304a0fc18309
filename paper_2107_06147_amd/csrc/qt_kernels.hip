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
#include "qt_device.hpp"
#include "qt_internal.h"

namespace qt {

// FP32 exp(x) - 1 without branches: the Taylor series to x^8 on |x| < 1/2
// (remainder < 2e-8 relative), exp2 - 1 elsewhere (there |result| > 0.39 and
// the absolute error of exp2 is a relative error ~1e-7).
__device__ __forceinline__ float qexpm1(float x)
{
    float p = 1.0f / 40320.0f;
    p = fmaf(p, x, 1.0f / 5040.0f);
    p = fmaf(p, x, 1.0f / 720.0f);
    p = fmaf(p, x, 1.0f / 120.0f);
    p = fmaf(p, x, 1.0f / 24.0f);
    p = fmaf(p, x, 1.0f / 6.0f);
    p = fmaf(p, x, 0.5f);
    p = fmaf(p, x, 1.0f);
    p = p * x;
    const float e = __builtin_amdgcn_exp2f(x * 1.44269504088896341f) - 1.0f;
    return fabsf(x) < 0.5f ? p : e;
}
__device__ __forceinline__ double qexpm1(double x) { return expm1(x); }

// FP32 sin and cos without branches: reduction by multiples of pi/2 with a
// two-constant (Cody-Waite) split of pi/2, then the Taylor series of sin to
// f^9 and cos to f^10 on |f| <= pi/4 (remainders < 2e-9).  Meant for the
// moderate arguments of the thermal phase (|x| < 1e4).
__device__ __forceinline__ void qsincos(float x, float* s, float* c)
{
    const float k = rintf(x * 0.636619772367581343f);
    float f = fmaf(-k, 1.57079637050628662109375f, x);
    f = fmaf(-k, -4.37113900018624283e-8f, f);
    const float f2 = f * f;
    float sp = -1.0f / 362880.0f;
    sp = fmaf(sp, f2, 1.0f / 5040.0f);
    sp = fmaf(sp, f2, -1.0f / 120.0f);
    sp = fmaf(sp, f2, 1.0f / 6.0f);
    sp = fmaf(-sp * f2, f, f);
    float cp = -1.0f / 3628800.0f;
    cp = fmaf(cp, f2, 1.0f / 40320.0f);
    cp = fmaf(cp, f2, -1.0f / 720.0f);
    cp = fmaf(cp, f2, 1.0f / 24.0f);
    cp = fmaf(cp, f2, -0.5f);
    cp = fmaf(cp, f2, 1.0f);
    const int q = (int)k & 3;
    const float ss = (q & 1) ? cp : sp, cc = (q & 1) ? sp : cp;
    *s = (q & 2) ? -ss : ss;
    *c = ((q + 1) & 2) ? -cc : cc;
}
__device__ __forceinline__ void qsincos(double x, double* s, double* c) { sincos(x, s, c); }

// kappa_hat at temperature T: the constant kappa_hat >= 0, or, for -1, -2,
// -3, the central, lower and upper fits to lattice data of the appendix
// "Munich potential", 1 / (a x^{3/2} + b x + c x^{1/2} + d) with
// x = T / T_c, T_c = 155 MeV; 0 where that denominator is not positive
// (below the fits' range).  Evaluated once per step, in FP64.
__device__ __forceinline__ double kappa_hat_at(double kappa_hat, double T)
{
    if (kappa_hat >= 0.0) return kappa_hat;
    const int k = (int)(-kappa_hat);
    const double a = k == 1 ? 0.00397 : k == 2 ? 0.00712 : 0.00272;
    const double b = k == 1 ? -0.08341 : k == 2 ? -0.14262 : -0.05854;
    const double c = k == 1 ? 0.98031 : k == 2 ? 1.55601 : 0.71513;
    const double d = k == 1 ? -0.51889 : k == 2 ? -0.80712 : -0.38197;
    const double x = T / 0.155;
    const double sx = sqrt(x);
    const double den = a * x * sx + b * x + c * sx + d;
    return den > 0.0 ? 1.0 / den : 0.0;
}

// Sum of K values over the workgroup, every lane receives all K sums.
template <int W, int K>
__device__ __forceinline__ void block_sum_vec(double* x, double* red)
{
#pragma unroll
    for (int i = 0; i < K; ++i) x[i] = wave_sum(x[i]);
    if constexpr (W > 64) {
        const int wave = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
#pragma unroll
            for (int i = 0; i < K; ++i) red[i * (W / 64) + wave] = x[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < K; ++i) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < W / 64; ++w) s += red[i * (W / 64) + w];
            x[i] = s;
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < K; ++i) x[i] = uniform(x[i]);
}

// exp(-i (dt/2) [V_coulomb(r) + l(l+1)/(M r^2)]): the time-independent part
// of the half-step factor (appendix "Munich potential").  The host computes
// it in FP64 for every (l, colour) with l <= l_tab, shared by all
// trajectories of a grid; a half-step reads the row of its (l, colour) (L1/L2
// resident: few rows are in use at a time).
template <class R, int N>
__device__ __forceinline__ const cx<R>* phase_row(const GroupDesc& g, int l, int c)
{
    return static_cast<const cx<R>*>(g.phase) + (size_t)(2 * l + c) * N;
}

// FP32 exp(x) - 1 on |x| <= 1/2: the Taylor series to x^8 (remainder
// < 2e-8 relative).  FP64 uses the library function.
__device__ __forceinline__ float expm1_small(float x)
{
    float p = 1.0f / 40320.0f;
    p = fmaf(p, x, 1.0f / 5040.0f);
    p = fmaf(p, x, 1.0f / 720.0f);
    p = fmaf(p, x, 1.0f / 120.0f);
    p = fmaf(p, x, 1.0f / 24.0f);
    p = fmaf(p, x, 1.0f / 6.0f);
    p = fmaf(p, x, 0.5f);
    p = fmaf(p, x, 1.0f);
    return p * x;
}
__device__ __forceinline__ double expm1_small(double x) { return expm1(x); }

// FP32 sin and cos on |x| <= pi/4: Taylor series to x^9 and x^10
// (remainders < 2e-9).  FP64 uses the library function.
__device__ __forceinline__ void sincos_small(float x, float* s, float* c)
{
    const float x2 = x * x;
    float sp = -1.0f / 362880.0f;
    sp = fmaf(sp, x2, 1.0f / 5040.0f);
    sp = fmaf(sp, x2, -1.0f / 120.0f);
    sp = fmaf(sp, x2, 1.0f / 6.0f);
    *s = fmaf(-sp * x2, x, x);
    float cp = -1.0f / 3628800.0f;
    cp = fmaf(cp, x2, 1.0f / 40320.0f);
    cp = fmaf(cp, x2, -1.0f / 720.0f);
    cp = fmaf(cp, x2, 1.0f / 24.0f);
    cp = fmaf(cp, x2, -0.5f);
    *c = fmaf(cp, x2, 1.0f);
}
__device__ __forceinline__ void sincos_small(double x, double* s, double* c) { sincos(x, s, c); }

// The half-step factor exp(-i V_eff(r_m) dt/2) of one time step is
//   P_m exp(z r_m^2),   z = zr + i zi = -(dt/2) c (kappa + i gamma) T^3,
// c = 1/2 (singlet) or 7/32 (octet), P_m the static phase (table row).  It is
// applied as two diagonal factors: the real damping D_m = exp(zr r_m^2),
// applied as u + (D_m - 1) u with D_m - 1 from expm1 so that its rounding is
// relative to the (small) difference and does not bias the norm step after
// step, and the phase C_m = P_m exp(i zi r_m^2), of modulus one.  The step is
//   D C [DST kin DST] C D,
// the bracket and C are unitary.  FP32-bulk renormalises C [DST kin DST] C
// as a whole to the norm it receives, which also absorbs the modulus error of
// C_m in FP32.  FAST: every argument is small (|zr| r^2 <= 1/2, |zi| r^2 <=
// pi/4 on the whole grid: a per-step, wave-uniform decision), so short
// series suffice.
template <class R, bool GAMMA, bool FAST>
struct HalfStep {
    const cx<R>* row;
    R dr, zr, zi;
    __device__ __forceinline__ R r2(int m) const
    {
        const R rm = R(m) * dr;
        return rm * rm;
    }
    __device__ __forceinline__ R em1(R x2) const
    {
        return FAST ? expm1_small(zr * x2) : qexpm1(zr * x2);
    }
    __device__ __forceinline__ cx<R> static_phase(int m) const { return ldg(row, m); }
    __device__ __forceinline__ cx<R> phase(cx<R> p, R x2) const
    {
        if constexpr (GAMMA) {
            R s, c;
            if constexpr (FAST) sincos_small(zi * x2, &s, &c);
            else qsincos(zi * x2, &s, &c);
            return p * mk(c, s);
        } else {
            return p;
        }
    }
};

// First half-step: u <- C D u.  Returns this lane's part of sum |D u|^2 (the
// norm the unitary block receives) when SUM; stores C_m in `fac` (this
// lane's slots, no other lane reads them) when CACHE, and D_m - 1 in dm
// (registers, for the second half-step).
template <class R, int N, int W, bool GAMMA, bool FAST, bool CACHE, bool SUM>
__device__ __forceinline__ double first_half(cx<R>* a, cx<R>* b, const HalfStep<R, GAMMA, FAST>& h,
                                             const Lanes<N, W>& ln, cx<R>* fac, R* dm)
{
    constexpr int R1 = Plan<N, W>::R1, T = Plan<N, W>::T;
    double acc = 0.0;
    cx<R>* mine = fac + ln.t;
    // static phases first: every load in flight at once
    cx<R> pr[2 * R1];
    sfor<0, R1>([&](auto Rr) QT_INL {
        pr[Rr] = h.static_phase(ln.ja + Rr * T);
        pr[R1 + Rr] = h.static_phase(ln.jb + Rr * T);
    });
    auto apply = [&](int m, cx<R>& u, auto E) QT_INL {
        const R x2 = h.r2(m);
        dm[E] = h.em1(x2);
        const cx<R> w = u + scale(u, dm[E]);
        if constexpr (SUM) acc += abs2d(w);
        const cx<R> C = h.phase(pr[E], x2);
        if constexpr (CACHE) mine[E * W] = C;
        u = C * w;
    };
    sfor<0, R1>([&](auto Rr) QT_INL {
        apply(ln.ja + Rr * T, a[Rr], std::integral_constant<int, Rr>{});
        apply(ln.jb + Rr * T, b[Rr], std::integral_constant<int, R1 + Rr>{});
        if constexpr ((Rr & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    });
    return acc;
}

// Second half-step: u <- D C u.  Adds this lane's sum |C u|^2 to x0 (when
// SUM0) and sum |D C u|^2 to x1.
template <class R, int N, int W, bool GAMMA, bool FAST, bool CACHE, bool SUM0>
__device__ __forceinline__ void second_half(cx<R>* a, cx<R>* b, const HalfStep<R, GAMMA, FAST>& h,
                                            const Lanes<N, W>& ln, const cx<R>* fac, const R* dm,
                                            double& x0, double& x1)
{
    constexpr int R1 = Plan<N, W>::R1, T = Plan<N, W>::T;
    const cx<R>* mine = fac + ln.t;
    auto apply = [&](int m, cx<R>& u, auto E) QT_INL {
        cx<R> C;
        if constexpr (CACHE) C = mine[E * W];
        else C = h.phase(h.static_phase(m), h.r2(m));
        const cx<R> w = C * u;
        if constexpr (SUM0) x0 += abs2d(w);
        u = w + scale(w, dm[E]);
        x1 += abs2d(u);
    };
    sfor<0, R1>([&](auto Rr) QT_INL {
        apply(ln.ja + Rr * T, a[Rr], std::integral_constant<int, Rr>{});
        apply(ln.jb + Rr * T, b[Rr], std::integral_constant<int, R1 + Rr>{});
        if constexpr ((Rr & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    });
}

// Calls f(GAMMA, FAST) with the two decisions as compile-time constants (the
// decisions are wave-uniform: one scalar branch).
template <class F>
__device__ __forceinline__ void with_factor_kind(bool gamma, bool fast, F&& f)
{
    using T_ = std::true_type;
    using F_ = std::false_type;
    if (gamma) {
        if (fast) f(T_{}, T_{});
        else f(T_{}, F_{});
    } else {
        if (fast) f(F_{}, T_{});
        else f(F_{}, F_{});
    }
}

// u <- u + f u (f small: a relative correction)
template <class R, int N, int W>
__device__ __forceinline__ void add_scaled(cx<R>* a, cx<R>* b, R f)
{
    constexpr int R1 = Plan<N, W>::R1;
    sfor<0, R1>([&](auto Rr) QT_INL {
        a[Rr] = a[Rr] + scale(a[Rr], f);
        b[Rr] = b[Rr] + scale(b[Rr], f);
    });
}

template <class R, int N, int W>
__device__ __forceinline__ double sum_abs2(const cx<R>* a, const cx<R>* b)
{
    constexpr int R1 = Plan<N, W>::R1;
    double acc = 0.0;
    sfor<0, R1>([&](auto Rr) QT_INL { acc += abs2d(a[Rr]) + abs2d(b[Rr]); });
    return acc;
}

// Writes the results of a finished trajectory (overlaps in FP64).
template <class R, int N, int W>
__device__ __forceinline__ void write_results(const GroupDesc& g, int64_t idx, const cx<R>* a,
                                              const cx<R>* b, const Lanes<N, W>& ln, double* red,
                                              int l, int c, int n_jumps, int status, int64_t steps,
                                              double norm, double first_r, double min_gap)
{
    constexpr int R1 = Plan<N, W>::R1, T = Plan<N, W>::T;
    // x[0..11]: re/im of the six dot products, x[12]: sum |u|^2, x[13]: sum r |u|^2
    double x[14];
#pragma unroll
    for (int i = 0; i < 14; ++i) x[i] = 0.0;
    const double* basis = g.basis;
    auto acc = [&](int m, cx<R> u) QT_INL {
        const double ur = (double)u.re, ui = (double)u.im;
        const double w2 = ur * ur + ui * ui;
        x[12] += w2;
        x[13] += (double)m * g.dr * w2;
#pragma unroll
        for (int bb = 0; bb < 6; ++bb) {
            const double ph = basis[bb * N + m];
            x[2 * bb] += ph * ur;
            x[2 * bb + 1] += ph * ui;
        }
    };
    // one element at a time: the scheduler would otherwise issue every basis
    // load at once and hold them all in registers
    sfor<0, R1>([&](auto Rr) QT_INL {
        acc(ln.ja + Rr * T, a[Rr]);
        __builtin_amdgcn_sched_barrier(0);
        acc(ln.jb + Rr * T, b[Rr]);
        __builtin_amdgcn_sched_barrier(0);
    });
    block_sum_vec<W, 14>(x, red);
    if (threadIdx.x == 0) {
        const qt_results& o = g.out;
        constexpr int basis_l[6] = {0, 0, 1, 0, 1, 2};
        const double nrm = x[12];
#pragma unroll
        for (int bb = 0; bb < 6; ++bb) {
            double ov = 0.0, sv = 0.0;
            if ((status == QT_TRAJ_OK || status == QT_TRAJ_NOJUMP) && c == QT_SINGLET &&
                l == basis_l[bb] && nrm > 0.0) {
                const double dr_ = g.dr * x[2 * bb], di_ = g.dr * x[2 * bb + 1];
                ov = (dr_ * dr_ + di_ * di_) / (g.dr * nrm);
                sv = g.init_overlap[bb] != 0.0 ? ov / g.init_overlap[bb] : ov;
            }
            if (o.overlap) o.overlap[6 * idx + bb] = ov;
            if (o.survival) o.survival[6 * idx + bb] = sv;
        }
        if (o.norm) o.norm[idx] = norm;
        if (o.first_r) o.first_r[idx] = first_r;
        if (o.mean_r) o.mean_r[idx] = nrm > 0.0 ? x[13] / nrm : 0.0;
        if (o.l) o.l[idx] = l;
        if (o.color) o.color[idx] = c;
        if (o.n_jumps) o.n_jumps[idx] = n_jumps;
        if (o.status) o.status[idx] = status;
        if (o.steps_done) o.steps_done[idx] = steps;
        if (o.min_gap) o.min_gap[idx] = min_gap;
    }
    if (g.out.psi) {
        double* dst = g.out.psi + (size_t)idx * 2 * N;
        sfor<0, R1>([&](auto Rr) QT_INL {
            const int ma = ln.ja + Rr * T, mb = ln.jb + Rr * T;
            dst[2 * ma] = (double)a[Rr].re;
            dst[2 * ma + 1] = (double)a[Rr].im;
            dst[2 * mb] = (double)b[Rr].re;
            dst[2 * mb + 1] = (double)b[Rr].im;
            __builtin_amdgcn_sched_barrier(0);
        });
    }
}

// Results of a trajectory that cannot jump: those of the batch's zeroth
// trajectory (paper: Sec. "Summary of QTraj execution", step 4, r_0 < rMin),
// with its own first threshold r and gap r_min - r (its gap to every norm of
// that evolution, the smallest being at the smallest norm).  The zeroth
// trajectory runs as the first item of the same launch; a trajectory that
// starts before it has finished is evolved instead, with the same results
// (see the label at completion).
template <int N, int W>
__device__ __forceinline__ void take_zeroth(const GroupDesc& g, int64_t idx, double r, double r_min)
{
    const qt_results& z = g.zeroth;
    const qt_results& o = g.out;
    if (threadIdx.x == 0) {
        if (o.norm) o.norm[idx] = z.norm[0];
        if (o.first_r) o.first_r[idx] = r;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            if (o.overlap) o.overlap[6 * idx + q] = z.overlap[q];
            if (o.survival) o.survival[6 * idx + q] = z.survival[q];
        }
        if (o.mean_r) o.mean_r[idx] = z.mean_r[0];
        if (o.l) o.l[idx] = z.l[0];
        if (o.color) o.color[idx] = z.color[0];
        if (o.n_jumps) o.n_jumps[idx] = 0;
        if (o.status) o.status[idx] = QT_TRAJ_NOJUMP;
        if (o.steps_done) o.steps_done[idx] = z.steps_done[0];
        if (o.min_gap) o.min_gap[idx] = r_min - r;
    }
    if (o.psi) {
        double* dst = o.psi + (size_t)idx * 2 * N;
        for (int m = threadIdx.x; m < 2 * N; m += W) dst[m] = z.psi[m];
    }
}

// ------------------------------------------------------------ FUSED -------

template <class R, int N, int W>
__global__ __launch_bounds__(W) void fused_kernel(FusedArgs A)
{
    using PL = Plan<N, W>;
    constexpr int R1 = PL::R1, T = PL::T;
    // FP32-bulk renormalises the unitary block of every step (see below)
    constexpr bool kRenorm = std::is_same<R, float>::value;
    __shared__ cx<R> buf[padded_len<N>()];
    __shared__ cx<R> wsum[W / 64];
    __shared__ double red[14 * (W / 64)];
    __shared__ int s_item;
    __shared__ int s_zdone;
    // per-lane cache of the phase factors C_m between the two half-steps of a
    // step, kept when it still leaves room for two workgroups per CU
    constexpr bool kCache =
        sizeof(cx<R>) * (padded_len<N>() + N) <= 80u * 1024u;
    __shared__ cx<R> fac[kCache ? N : 1];

    const Lanes<N, W> ln(threadIdx.x);
    const cx<R>* tw = static_cast<const cx<R>*>(A.tw);
    const cx<R>* prew = static_cast<const cx<R>*>(A.prew);

    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(A.queue, 1);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (item >= A.n_items) break;
        const GroupDesc& g = A.groups[uniform(A.item_group[item])];
        const int64_t idx = uniform(A.item_index[item]);
        const uint64_t stride = g.traj_id_stride ? g.traj_id_stride : 1u;
        const uint64_t traj_id = g.traj_id0 + (uint64_t)idx * stride;
        const Kin<R>* kin = static_cast<const Kin<R>*>(g.kin);

        cx<R> a[R1], b[R1];
        int l, c, n_jumps, status;
        int64_t step;
        double r, first_r, min_gap, norm;
        const bool resume = g.st != nullptr && g.st[idx].started;
        if (resume) {
            const TrajState s = g.st[idx];
            if (s.done) continue;
            const cx<R>* src = static_cast<const cx<R>*>(g.st_psi) + (size_t)idx * N;
            sfor<0, R1>([&](auto Rr) QT_INL {
                a[Rr] = src[ln.ja + Rr * T];
                b[Rr] = src[ln.jb + Rr * T];
            });
            l = s.l; c = s.c; n_jumps = s.n_jumps; status = s.status; step = s.step;
            r = s.r; first_r = s.first_r; min_gap = s.min_gap; norm = s.norm;
        } else {
            // the zeroth trajectory of a batch has threshold 0: it never jumps
            const U4 e0 = event_block(g.seed, traj_id, 0);
            r = uniform(g.flags & kFlagZeroth ? 0.0 : uniform01(e0.w[2]));
            if (g.zeroth.norm != nullptr) {
                // has the batch's zeroth trajectory finished?  One decision
                // for the whole workgroup, then each lane's own acquire
                if (threadIdx.x == 0)
                    s_zdone = __hip_atomic_load(g.zdone, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                __syncthreads();
                const int zd = __builtin_amdgcn_readfirstlane(s_zdone);
                __syncthreads();
                if (zd) {
                    (void)__hip_atomic_load(g.zdone, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                    const double r_min = uniform(g.zeroth.min_gap[0]);
                    if (r < r_min) {
                        // below every norm of the no-jump evolution: this
                        // trajectory is that evolution
                        take_zeroth<N, W>(g, idx, r, r_min);
                        continue;
                    }
                }
            }
            sfor<0, R1>([&](auto Rr) QT_INL {
                const int ma = ln.ja + Rr * T, mb = ln.jb + Rr * T;
                a[Rr] = mk(R(g.init_psi[2 * ma]), R(g.init_psi[2 * ma + 1]));
                b[Rr] = mk(R(g.init_psi[2 * mb]), R(g.init_psi[2 * mb + 1]));
                if constexpr ((Rr & 3) == 3) __builtin_amdgcn_sched_barrier(0);
            });
            l = g.init_l; c = g.init_color; n_jumps = 0; status = QT_TRAJ_OK; step = 0;
            min_gap = __builtin_huge_val();
            first_r = r;
            norm = g.dr * block_sum<W>(sum_abs2<R, N, W>(a, b), red);
            if (g.do_jumps && r > g.r_max) status = QT_TRAJ_RMAX;
        }

        // every per-trajectory scalar is identical on all lanes: say so
        l = uniform(l); c = uniform(c); n_jumps = uniform(n_jumps); status = uniform(status);
        step = uniform(step); r = uniform(r); norm = uniform(norm);
        int64_t end = uniform(g.n_steps);
        if (A.seg_steps > 0 && step + A.seg_steps < end) end = step + A.seg_steps;
        if (l > g.l_tab) status = QT_TRAJ_LMAX;
        const bool has_gamma = g.gamma_hat != 0.0;
        const R dr = R(g.dr);
        const double xmax = (double)(N - 1) * g.dr * (double)(N - 1) * g.dr;
        int cur = 0;
        while (status == QT_TRAJ_OK && step < end) {
            // lane-derived values are recomputed every step (see opaque_lane)
            const Lanes<N, W> ls(opaque_lane(threadIdx.x));
            const int64_t n = step;
            const double t = g.tau_start + (double)n * g.dt;
            const double Tn = temperature_at(g.tau, g.Ttab, g.n_tab, t, cur);
            const double T3 = Tn * Tn * Tn;
            const double cc = (c == QT_SINGLET) ? 0.5 : 7.0 / 32.0;
            const double kh = kappa_hat_at(g.kappa_hat, Tn);
            const R zr = R(-0.5 * g.dt * cc * kh * T3);
            const R zi = R(-0.5 * g.dt * cc * g.gamma_hat * T3);
            const cx<R>* row = opaque(phase_row<R, N>(g, l, c));
            // FP64 always takes the library functions
            const bool fast = !kRenorm || (fabs(-0.5 * g.dt * cc * kh * T3) * xmax <= 0.5 &&
                                           fabs(-0.5 * g.dt * cc * g.gamma_hat * T3) * xmax <= 0.78);

            cx<R> pw[Plan<N, W>::R1];
            load_prew<R, N, W>(pw, prew, ls);
            R dm[Plan<N, W>::P];
            double n_in = 0.0;
            with_factor_kind(has_gamma, fast, [&](auto G, auto F) QT_INL {
                const HalfStep<R, G, F> h{row, dr, zr, zi};
                n_in = first_half<R, N, W, G, F, kCache, kRenorm>(a, b, h, ls, fac, dm);
            });
            const cx<R>* tw_n = opaque(tw);
            dst1<R, N, W, true>(a, b, pw, prew, ls, buf, wsum, tw_n, kin);
            dst1<R, N, W, false>(a, b, pw, prew, ls, buf, wsum, opaque(tw_n), nullptr);
            // x: sum |D u|^2 after the first half-step (the norm the unitary
            // block receives), sum |C u|^2 (what it returns), sum |D C u|^2
            double x[3] = {n_in, 0.0, 0.0};
            with_factor_kind(has_gamma, fast, [&](auto G, auto F) QT_INL {
                const HalfStep<R, G, F> h{opaque(row), dr, zr, zi};
                second_half<R, N, W, G, F, kCache, kRenorm>(a, b, h, ls, fac, dm, x[1], x[2]);
            });
            if constexpr (kRenorm) {
                // the block C DST kin DST C is unitary: restore the norm it
                // received (D commutes with the scaling)
                block_sum_vec<W, 3>(x, red);
                add_scaled<R, N, W>(a, b, R(sqrt(x[0] / x[1]) - 1.0));
                norm = g.dr * x[2] * (x[0] / x[1]);
            } else {
                norm = g.dr * block_sum<W>(x[2], red);
            }
            step = n + 1;
            if (!g.do_jumps) continue;
            const double gap = fabs(norm - r);
            if (gap < min_gap) min_gap = gap;
            if (norm <= r) {
                if (g.max_jumps >= 0 && n_jumps >= g.max_jumps) {
                    status = QT_TRAJ_MAXJUMPS;
                    break;
                }
                const U4 e = event_block(g.seed, traj_id, (int64_t)n_jumps + 1);
                const double ul = uniform01(e.w[0]), uc = uniform01(e.w[1]);
                l = (ul < (double)l / (double)(2 * l + 1)) ? l - 1 : l + 1;
                c = (c == QT_OCTET) ? (uc < 2.0 / 7.0 ? QT_SINGLET : QT_OCTET) : QT_OCTET;
                sfor<0, R1>([&](auto Rr) QT_INL {
                    a[Rr] = scale(a[Rr], R(ls.ja + Rr * T) * dr);
                    b[Rr] = scale(b[Rr], R(ls.jb + Rr * T) * dr);
                });
                const double s2 = g.dr * block_sum<W>(sum_abs2<R, N, W>(a, b), red);
                const R f = R(1.0 / sqrt(s2));
                sfor<0, R1>([&](auto Rr) QT_INL {
                    a[Rr] = scale(a[Rr], f);
                    b[Rr] = scale(b[Rr], f);
                });
                norm = g.dr * block_sum<W>(sum_abs2<R, N, W>(a, b), red);
                r = uniform(uniform01(e.w[2]));
                n_jumps += 1;
                l = uniform(l);
                c = uniform(c);
                if (l > g.l_tab) {
                    status = QT_TRAJ_LMAX;
                    break;
                }
            }
        }
        const bool done = status != QT_TRAJ_OK || step >= g.n_steps;
        if (done) {
            // in a batch with the no-jump shortcut, a trajectory that ran to
            // the end without a jump evolved exactly as the zeroth one: its
            // threshold lies below every norm of that evolution
            if (g.zeroth.norm != nullptr && status == QT_TRAJ_OK && n_jumps == 0)
                status = QT_TRAJ_NOJUMP;
            write_results<R, N, W>(g, idx, a, b, ln, red, l, c, n_jumps, status, step, norm,
                                   first_r, min_gap);
            if (g.flags & kFlagZeroth) {
                // publish: every lane's writes first, then the flag
                __threadfence();
                __syncthreads();
                if (threadIdx.x == 0)
                    __hip_atomic_store(g.zdone, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (g.st) {
            // checkpoint (the final state too, so a job can return it)
            {
                cx<R>* dst = static_cast<cx<R>*>(g.st_psi) + (size_t)idx * N;
                sfor<0, R1>([&](auto Rr) QT_INL {
                    dst[ln.ja + Rr * T] = a[Rr];
                    dst[ln.jb + Rr * T] = b[Rr];
                });
            }
            if (threadIdx.x == 0) {
                TrajState s;
                s.step = step; s.l = l; s.c = c; s.n_jumps = n_jumps; s.status = status;
                s.started = 1; s.done = done ? 1 : 0; s.pad0 = 0; s.pad1 = 0;
                s.r = r; s.first_r = first_r; s.min_gap = min_gap; s.norm = norm;
                g.st[idx] = s;
            }
        }
    }
}

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

template <class R, int N, int W>
hipError_t launch_fused(const FusedArgs& a, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((fused_kernel<R, N, W>), dim3(grid), dim3(W), 0, s, a);
    return hipGetLastError();
}

template <class R, int N, int W>
int occupancy_fused()
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fused_kernel<R, N, W>, W, 0) !=
        hipSuccess)
        return 0;
    return blocks;
}

struct FusedEntry {
    int prec, N, W;
    fused_launcher launch;
    int (*occ)();
};

#define QT_F32(N, W) {QT_FP32_BULK, N, W, launch_fused<float, N, W>, occupancy_fused<float, N, W>}
#define QT_F64(N, W) {QT_FP64, N, W, launch_fused<double, N, W>, occupancy_fused<double, N, W>}

static const FusedEntry kFused[] = {
    // FP32-bulk: 4..16 complex values per lane
    QT_F32(256, 64),   QT_F32(512, 64),   QT_F32(1024, 64),  QT_F32(1024, 128),
    QT_F32(1024, 256), QT_F32(2048, 128), QT_F32(2048, 256), QT_F32(2048, 512),
    QT_F32(4096, 256), QT_F32(4096, 512), QT_F32(4096, 1024), QT_F32(8192, 512),
    QT_F32(8192, 1024),
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
    // loadSpaceKernel(T_n): exp(-i V_eff dt/2) from the full potential
    const double T = g.Tn[n];
    const double T3 = T * T * T;
    const double r = (double)m * g.dr;
    const double cent = (double)s.l * (double)(s.l + 1) / (g.mass * r * r);
    double VR, VI;
    if (s.c == QT_SINGLET) {
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
        s.norm = nrm; s.started = 1; s.pad0 = 0; s.pad1 = 0;
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
                sv = g.init_overlap[bb] != 0.0 ? ov / g.init_overlap[bb] : ov;
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
