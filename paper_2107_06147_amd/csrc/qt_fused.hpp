// qt_fused.hpp -- the fused persistent kernel of the quantum-trajectory
// solver and its per-step building blocks (half-step factors of the Munich
// and the isotropic KSU potentials, the FP32 elementary functions, the
// shortcut copy, the results).  Instantiated per (precision, N, W,
// potential) by qt_kernels.hip (Munich) and qt_kernels_ksu.hip (KSU).
#pragma once
#include "qt_device.hpp"
#include "qt_dst32.hpp"
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

// FP32 sin(x) and cos(x) - 1, the same reduction and series as qsincos, with
// cos - 1 formed without adding 1 on the first quadrant: a phase factor of
// small angle keeps its full relative accuracy in this form (cos x itself
// rounds to 1 or 1 - 2^-24 there, a bias in the modulus of about x^2/2).
__device__ __forceinline__ void qsincos_m1(float x, float* s, float* cm1)
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
    const float cpm1 = cp * f2;                 // cos f - 1
    const int q = (int)k & 3;
    // q = 0: (sin, cos-1) = (sp, cpm1); 1: (cp, -sp - 1); 2: (-sp, -2 - cpm1);
    // 3: (-cp, sp - 1), with cp = 1 + cpm1
    const float c1 = 1.0f + cpm1;
    *s = q == 0 ? sp : q == 1 ? c1 : q == 2 ? -sp : -c1;
    *cm1 = q == 0 ? cpm1 : q == 1 ? -sp - 1.0f : q == 2 ? -2.0f - cpm1 : sp - 1.0f;
}

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
// resident: few rows are in use at a time).  FP32 rows hold the factor minus
// one (see apply_phase), in mirror pairs (see load_mirror_pairs).
template <class R, int N>
__device__ __forceinline__ const cx<R>* phase_row(const GroupDesc& g, int l, int c)
{
    return static_cast<const cx<R>*>(g.phase) + (size_t)(2 * l + c) * N;
}

// FP32 exp(x) - 1 on |x| <= 1/2: the Taylor series to x^8 (remainder
// < 2e-8 relative); FP64 to x^15 (remainder < 5e-17 relative, two units of
// the FP64 roundoff in all).
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
__device__ __forceinline__ double expm1_small(double x)
{
    double p = 1.0 / 1307674368000.0;                     // 1/15!
    p = fma(p, x, 1.0 / 87178291200.0);                   // 1/14!
    p = fma(p, x, 1.0 / 6227020800.0);                    // 1/13!
    p = fma(p, x, 1.0 / 479001600.0);                     // 1/12!
    p = fma(p, x, 1.0 / 39916800.0);                      // 1/11!
    p = fma(p, x, 1.0 / 3628800.0);                       // 1/10!
    p = fma(p, x, 1.0 / 362880.0);                        // 1/9!
    p = fma(p, x, 1.0 / 40320.0);                         // 1/8!
    p = fma(p, x, 1.0 / 5040.0);                          // 1/7!
    p = fma(p, x, 1.0 / 720.0);                           // 1/6!
    p = fma(p, x, 1.0 / 120.0);                           // 1/5!
    p = fma(p, x, 1.0 / 24.0);                            // 1/4!
    p = fma(p, x, 1.0 / 6.0);                             // 1/3!
    p = fma(p, x, 0.5);                                   // 1/2!
    p = fma(p, x, 1.0);
    return p * x;
}

// FP32 sin and cos on |x| <= pi/4: Taylor series to x^9 and x^10
// (remainders < 2e-9).
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
// FP64 sin and cos on |x| <= pi/4: Taylor series to x^17 and x^18
// (remainders below 2e-19 and 5e-21 there), cheaper than the library
// functions' range reduction.
__device__ __forceinline__ void sincos_small(double x, double* s, double* c)
{
    const double x2 = x * x;
    double sp = 1.0 / 355687428096000.0;                  // 1/17!
    sp = fma(sp, -x2, 1.0 / 1307674368000.0);             // 1/15!
    sp = fma(sp, -x2, 1.0 / 6227020800.0);                // 1/13!
    sp = fma(sp, -x2, 1.0 / 39916800.0);                  // 1/11!
    sp = fma(sp, -x2, 1.0 / 362880.0);                    // 1/9!
    sp = fma(sp, -x2, 1.0 / 5040.0);                      // 1/7!
    sp = fma(sp, -x2, 1.0 / 120.0);                       // 1/5!
    sp = fma(sp, -x2, 1.0 / 6.0);                         // 1/3!
    *s = fma(-sp * x2, x, x);
    double cp = 1.0 / 6402373705728000.0;                 // 1/18!
    cp = fma(cp, -x2, 1.0 / 20922789888000.0);            // 1/16!
    cp = fma(cp, -x2, 1.0 / 87178291200.0);               // 1/14!
    cp = fma(cp, -x2, 1.0 / 479001600.0);                 // 1/12!
    cp = fma(cp, -x2, 1.0 / 3628800.0);                   // 1/10!
    cp = fma(cp, -x2, 1.0 / 40320.0);                     // 1/8!
    cp = fma(cp, -x2, 1.0 / 720.0);                       // 1/6!
    cp = fma(cp, -x2, 1.0 / 24.0);                        // 1/4!
    cp = fma(cp, -x2, 0.5);                               // 1/2!
    *c = fma(-cp, x2, 1.0);
}

// FP32 sin(x) and cos(x) - 1 on |x| <= pi/4, cos - 1 without the 1 (see
// qsincos_m1).
__device__ __forceinline__ void sincos_small_m1(float x, float* s, float* cm1)
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
    *cm1 = cp * x2;
}

// A unit phase factor C applied to w.  FP64 holds C and multiplies.  FP32
// holds C - 1 (the host tables, the LDS cache and the per-step factors are
// all in this form) and forms w + (C - 1) w, whose only full-size rounding
// is the final addition: the modulus of C is then exact to the accuracy of
// the small C - 1 instead of carrying the bias of a rounded cos near 1,
// which is the same every step and grows the error linearly.
__device__ __forceinline__ cx<double> apply_phase(cx<double> w, cx<double> C) { return C * w; }
__device__ __forceinline__ cx<float> apply_phase(cx<float> w, cx<float> cm1)
{
    const float re = fmaf(cm1.re, w.re, -(cm1.im * w.im));
    const float im = fmaf(cm1.re, w.im, cm1.im * w.re);
    return mk(w.re + re, w.im + im);
}
// The product of two phase factors in the form apply_phase takes: C1 C2
// (FP64), (C1 - 1) + (C2 - 1) + (C1 - 1)(C2 - 1) (FP32).
__device__ __forceinline__ cx<double> phase_product(cx<double> a, cx<double> b) { return a * b; }
__device__ __forceinline__ cx<float> phase_product(cx<float> a, cx<float> b)
{
    return a + b + a * b;
}

// FP64 factors outside the series' ranges (a rare path: large time steps or
// temperatures): the library functions, in functions of their own so that
// their constants do not take registers in the time loop.
__device__ __noinline__ double expm1_far(double x) { return expm1(x); }
__device__ __noinline__ double2 sincos_far(double x)
{
    double s, c;
    sincos(x, &s, &c);
    return make_double2(s, c);
}

// The half-step factor exp(-i V_eff(r_m) dt/2) of one time step is
//   P_m exp(z r_m^2),   z = zr + i zi = -(dt/2) c (kappa + i gamma) T^3,
// c = 1/2 (singlet) or 7/32 (octet), P_m the static phase (table row).  It is
// applied as two diagonal factors: the real damping D_m = exp(zr r_m^2),
// applied as u + (D_m - 1) u with D_m - 1 from expm1 so that its rounding is
// relative to the (small) difference and does not bias the norm step after
// step, and the phase C_m = P_m exp(i zi r_m^2), of modulus one (held as
// C_m - 1 in FP32, apply_phase).  The step is
//   D C [DST kin DST] C D,
// the bracket and C are unitary.  FP32-bulk renormalises C [DST kin DST] C
// as a whole to the norm it receives, which also absorbs what modulus error
// of C_m remains in FP32.  FAST: every argument is small (|zr| r^2 <= 1/2, |zi| r^2 <=
// pi/4 on the whole grid: a per-step, wave-uniform decision), so short
// series suffice.
template <class R, bool GAMMA, bool FAST>
struct HalfStep {
    // without the thermal phase C_m is the static phase: the same every step
    // until a jump changes (l, colour), so a cache of it stays valid
    static constexpr bool kStaticC = !GAMMA;
    // FP32 rows hold mirror pairs (see load_mirror_pairs)
    static constexpr bool kPairRows = std::is_same<R, float>::value;
    const cx<R>* row;
    R dr, zr, zi;
    __device__ __forceinline__ R r2(int m) const
    {
        const R rm = R(m) * dr;
        return rm * rm;
    }
    __device__ __forceinline__ R em1(R x2) const
    {
        if constexpr (FAST) return expm1_small(zr * x2);
        else if constexpr (std::is_same<R, double>::value) return expm1_far(zr * x2);
        else return qexpm1(zr * x2);
    }
    __device__ __forceinline__ cx<R> static_phase(int m) const
    {
        static_assert(!kPairRows, "FP32 rows hold mirror pairs: read them with load_mirror_pairs");
        return ldg(row, m);
    }
    __device__ __forceinline__ cx<R> phase(cx<R> p, R x2) const
    {
        if constexpr (GAMMA) {
            R s, c;
            if constexpr (std::is_same<R, float>::value) {
                if constexpr (FAST) sincos_small_m1(zi * x2, &s, &c);
                else qsincos_m1(zi * x2, &s, &c);
            } else {
                if constexpr (FAST) {
                    sincos_small(zi * x2, &s, &c);
                } else {
                    const double2 sc = sincos_far(zi * x2);
                    s = sc.x;
                    c = sc.y;
                }
            }
            return phase_product(p, mk(c, s));
        } else {
            return p;
        }
    }
    // the interface of a half-step factor: data loaded ahead for point m,
    // then D_m - 1 and C_m
    __device__ __forceinline__ cx<R> preload(int m) const { return static_phase(m); }
    __device__ __forceinline__ void factors(int m, cx<R> pre, R& dm1, cx<R>& C) const
    {
        const R x2 = r2(m);
        dm1 = em1(x2);
        C = phase(pre, x2);
    }
    __device__ __forceinline__ R damping(int m) const { return em1(r2(m)); }
};

// The half-step factor of the isotropic KSU potential (appendix "Isotropic
// KSU potential"), computed per point from the step's Debye mass m_D and
// width coefficient c_I = alpha_s C_F T:
//   V_R = min(V_KMS, V_vac(r_SB)) + l(l+1)/(M r^2),
//   V_KMS = -(a/r)(1 + x) e^{-x} + 2 sigma r (1 - e^{-x})/x - sigma r e^{-x},
//   V_I = -c_I phi(x),  x = m_D r,
// D = exp(V_I dt/2), C = exp(-i V_R dt/2).  phi comes from a cubic Hermite
// table of (phi, phi') on [0, 1/2] (spacing 1/8192) and [1/2, 64] (spacing
// 1/256), and its asymptotic series beyond.  The point r = 0 (a boundary
// value, always 0) gets the factor 1.
constexpr double kKsuA = 0.409, kKsuSigma = 0.21;
constexpr int kPhiFine = 4096, kPhiCoarse = 16256;   // intervals
template <class R>
struct HalfStepKSU {
    static constexpr bool kStaticC = false;
    static constexpr bool kPairRows = false;
    const cx<R>* phi_tab;     // (phi, phi'): kPhiFine + 1 fine, then kPhiCoarse + 1
    R dr, half_dt, md, cI, cent, vsb;
    __device__ __forceinline__ cx<R> preload(int) const { return mk(R(0), R(0)); }
    __device__ __forceinline__ R phi(R x) const
    {
        auto herm = [](R t, cx<R> p0, cx<R> p1, R h) QT_INL {
            const R t2 = t * t, t3 = t2 * t;
            return (R(2) * t3 - R(3) * t2 + R(1)) * p0.re + (t3 - R(2) * t2 + t) * h * p0.im +
                   (R(3) * t2 - R(2) * t3) * p1.re + (t3 - t2) * h * p1.im;
        };
        if (x < R(0.5)) {
            const R s = x * R(kPhiFine * 2);
            const int i = (int)s;
            return herm(s - R(i), ldg(phi_tab, i), ldg(phi_tab, i + 1), R(1.0 / (kPhiFine * 2)));
        }
        if (x < R(64)) {
            const R s = (x - R(0.5)) * R(256);
            const int i = (int)s;
            const int k = kPhiFine + 1 + i;
            return herm(s - R(i), ldg(phi_tab, k), ldg(phi_tab, k + 1), R(1.0 / 256.0));
        }
        const R q = R(1) / (x * x);
        return R(1) - q * (R(2) + q * (R(8) + q * (R(144) + q * (R(5760) + q * R(403200)))));
    }
    __device__ __forceinline__ void factors(int m, cx<R>, R& dm1, cx<R>& C) const
    {
        const R r = R(m > 0 ? m : 1) * dr;
        const R x = md * r;
        const R e = exp(-x);
        const R q = x > R(1e-4) ? -qexpm1(-x) / x : R(1) - x * (R(0.5) - x * R(1.0 / 6.0));
        const R kms = -(R(kKsuA) / r) * (R(1) + x) * e + R(2 * kKsuSigma) * r * q - R(kKsuSigma) * r * e;
        const R vr = (kms <= vsb ? kms : vsb) + cent / (r * r);
        const R vi = -cI * phi(x);
        R s, c;
        dm1 = m > 0 ? qexpm1(half_dt * vi) : R(0);
        if constexpr (std::is_same<R, float>::value) {
            qsincos_m1(-half_dt * vr, &s, &c);       // c = cos - 1
            C = m > 0 ? mk(c, s) : mk(R(0), R(0));
        } else {
            qsincos(-half_dt * vr, &s, &c);
            C = m > 0 ? mk(c, s) : mk(R(1), R(0));
        }
    }
};

// Per-step scalars of the KSU potential at temperature T: the one-loop
// alpha_s(2 pi T) from alpha_s(5 GeV) = 0.2034 with 3 light flavours, the
// Debye mass m_D = F T sqrt(N_c (1 + N_F/6) pi (4/3) alpha_s) and c_I =
// alpha_s C_F T; no medium (0, 0) where T <= 0 or the coupling is not
// positive (at and below the one-loop pole).
__device__ __forceinline__ void ksu_medium(double T, double md_factor, double* md, double* cI)
{
    *md = 0.0;
    *cI = 0.0;
    if (!(T > 0.0)) return;
    const double pi = 3.14159265358979323846;
    const double inv = 1.0 / 0.2034 + (11.0 - 2.0) / (2.0 * pi) * log(2.0 * pi * T / 5.0);
    if (!(inv > 0.0)) return;
    const double as = 1.0 / inv;
    *md = md_factor * T * sqrt(3.0 * 1.5 * pi * (4.0 / 3.0) * as);
    *cI = as * (4.0 / 3.0) * T;
}

// The static phase row of (l, colour) into this lane's slots of the cache
// `fac` (slot E < R1: point ja + E T; slot R1 + E: point jb + E T).
template <class R, int N, int W>
__device__ __forceinline__ void fill_static_phase(cx<R>* fac, const cx<R>* row,
                                                  const Lanes<N, W>& ln)
{
    constexpr int R1 = Plan<N, W>::R1, T = Plan<N, W>::T;
    cx<R>* mine = fac + ln.t;
    if constexpr (std::is_same<R, float>::value) {
        cx<float> pr[2 * R1];
        load_mirror_pairs<N, W>(row, ln, pr);
        sfor<0, 2 * R1>([&](auto E) QT_INL { mine[E * W] = pr[E]; });
    } else {
        sfor<0, R1>([&](auto Rr) QT_INL {
            mine[Rr * W] = ldg(row, ln.ja + Rr * T);
            mine[(R1 + Rr) * W] = ldg(row, ln.jb + Rr * T);
        });
    }
}

// The damping factors of the slots (2g, 2g + 1, R1 + 2g, R1 + 2g + 1) of
// lane t as one 16-byte LDS entry, at dml[4 (t + g W)]: one LDS write and
// one read per four factors.
template <int W, class R>
__device__ __forceinline__ void store_dm4(R* dml, int t, int g, R d0, R d1, R d2, R d3)
{
    typedef R v4 __attribute__((ext_vector_type(4)));
    v4 v;
    v.x = d0;
    v.y = d1;
    v.z = d2;
    v.w = d3;
    reinterpret_cast<v4*>(dml)[t + g * W] = v;
}
template <int W, class R>
__device__ __forceinline__ void load_dm4(const R* dml, int t, int g, R* d)
{
    typedef R v4 __attribute__((ext_vector_type(4)));
    const v4 v = reinterpret_cast<const v4*>(dml)[t + g * W];
    d[0] = v.x;
    d[1] = v.y;
    d[2] = v.z;
    d[3] = v.w;
}

// First half-step: u <- C D u.  Returns this lane's part of sum |D u|^2 (the
// norm the unitary block receives) when SUM; D_m - 1 goes to dm (registers,
// for the second half-step), and with DML also to this lane's entries of the
// LDS array dml (store_dm4), from which the second half-step then reads it.
// With CACHE, C_m is in `fac` (this lane's slots, no other lane reads them)
// for the second half-step: stored here, or, for a static C (H::kStaticC)
// when STATIC, already there (fill_static_phase) and read from it instead
// of the table.
template <class R, int N, int W, class H, bool CACHE, bool SUM, bool STATIC = false,
          bool DML = false>
__device__ __forceinline__ double first_half(cx<R>* a, cx<R>* b, const H& h,
                                             const Lanes<N, W>& ln, cx<R>* fac, R* dm,
                                             R* dml = nullptr)
{
    constexpr int R1 = Plan<N, W>::R1, T = Plan<N, W>::T;
    constexpr bool kCached = CACHE && STATIC && H::kStaticC;
    double acc = 0.0;
    cx<R>* mine = fac + ln.t;
    // table (or cache) data first: every load in flight at once
    cx<R> pr[2 * R1];
    if constexpr (!kCached && H::kPairRows) {
        load_mirror_pairs<N, W>(h.row, ln, pr);
    } else {
        sfor<0, R1>([&](auto Rr) QT_INL {
            if constexpr (kCached) {
                pr[Rr] = mine[Rr * W];
                pr[R1 + Rr] = mine[(R1 + Rr) * W];
            } else {
                pr[Rr] = h.preload(ln.ja + Rr * T);
                pr[R1 + Rr] = h.preload(ln.jb + Rr * T);
            }
        });
    }
    auto apply = [&](int m, cx<R>& u, auto E) QT_INL {
        cx<R> C;
        if constexpr (kCached) {
            dm[E] = h.damping(m);
            C = pr[E];
        } else {
            h.factors(m, pr[E], dm[E], C);
            if constexpr (CACHE) mine[E * W] = C;
        }
        const cx<R> w = u + scale(u, dm[E]);
        if constexpr (SUM) add_abs2(acc, w);
        u = apply_phase(w, C);
    };
    sfor<0, R1>([&](auto Rr) QT_INL {
        constexpr int r = Rr;
        apply(ln.ja + r * T, a[r], std::integral_constant<int, r>{});
        apply(ln.jb + r * T, b[r], std::integral_constant<int, R1 + r>{});
        if constexpr (DML && (r & 1) == 1)
            store_dm4<W>(dml, ln.t, r / 2, dm[r - 1], dm[r], dm[R1 + r - 1], dm[R1 + r]);
        if constexpr ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    });
    return acc;
}

// Second half-step: u <- D C u.  Adds this lane's sum |C u|^2 to x0 (when
// SUM0) and sum |D C u|^2 to x1.  D_m - 1 comes from dm, with DML from the
// LDS entries first_half stored it in (load_dm4), with RECOMP from the
// factor itself (computed again as in first_half, the same value).
template <class R, int N, int W, class H, bool CACHE, bool SUM0, bool DML = false,
          bool RECOMP = false>
__device__ __forceinline__ void second_half(cx<R>* a, cx<R>* b, const H& h,
                                            const Lanes<N, W>& ln, const cx<R>* fac, const R* dm,
                                            double& x0, double& x1, const R* dml = nullptr)
{
    constexpr int R1 = Plan<N, W>::R1, T = Plan<N, W>::T;
    const cx<R>* mine = fac + ln.t;
    constexpr bool kPairs = !CACHE && H::kPairRows;
    cx<R> pr[kPairs ? 2 * R1 : 1];
    R dq[4];
    if constexpr (kPairs) load_mirror_pairs<N, W>(h.row, ln, pr);
    auto apply = [&](int m, cx<R>& u, auto E) QT_INL {
        cx<R> C;
        if constexpr (CACHE) {
            C = mine[E * W];
        } else {
            R unused;
            if constexpr (kPairs) h.factors(m, pr[E], unused, C);
            else h.factors(m, h.preload(m), unused, C);
        }
        const cx<R> w = apply_phase(u, C);
        if constexpr (SUM0) add_abs2(x0, w);
        if constexpr (DML) {
            constexpr int e = E;
            u = w + scale(w, dq[(e < R1 ? 0 : 2) + (e & 1)]);
        } else if constexpr (RECOMP) {
            u = w + scale(w, h.damping(m));
        } else {
            u = w + scale(w, dm[E]);
        }
        add_abs2(x1, u);
    };
    sfor<0, R1>([&](auto Rr) QT_INL {
        constexpr int r = Rr;
        if constexpr (DML && (r & 1) == 0) load_dm4<W>(dml, ln.t, r / 2, dq);
        apply(ln.ja + r * T, a[r], std::integral_constant<int, r>{});
        apply(ln.jb + r * T, b[r], std::integral_constant<int, R1 + r>{});
        if constexpr ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
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
    sfor<0, R1>([&](auto Rr) QT_INL {
        add_abs2(acc, a[Rr]);
        add_abs2(acc, b[Rr]);
    });
    return acc;
}

// Entry e (the e-th jump, 0-based) of trajectory idx's jump log: the step
// after which it happened and the new (l, colour).  Lane 0 writes.
__device__ __forceinline__ void log_jump(const qt_results& o, int64_t idx, int e, int64_t n, int l,
                                         int c)
{
    if (o.jump_log != nullptr && e < o.jump_log_cap && threadIdx.x == 0) {
        int32_t* d = o.jump_log + 3 * ((size_t)idx * o.jump_log_cap + e);
        d[0] = (int32_t)n;
        d[1] = l;
        d[2] = c;
    }
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
                // (an initial population below 1e-12 is rounding: no ratio)
                sv = g.init_overlap[bb] > 1e-12 ? ov / g.init_overlap[bb] : ov;
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

// The form of a fused kernel: its LDS and its occupancy target.
//
// Every kernel runs at least two waves per SIMD: the register budget is then
// 256 per lane (VGPRs and AGPRs together), so that the allocator never trades
// a register or two for half the occupancy.
//
// Lean form (Munich potential, workgroups of several waves, FP32 bulk with
// 16 values per lane or FP64 with 8): three waves per SIMD (168 registers).
// Its workgroup keeps no cache of the phase factors C_m (the second
// half-step reads the static phase again and recomputes the thermal one),
// does not keep the damping factors D_m - 1 in registers between the two
// half-steps (FP32 holds them in LDS; FP64 recomputes them, which its VALU
// has room for, and gives the LDS to the padding of its transforms instead),
// and runs the transforms' lean forms (kin_block32 LEAN, dst1 LATE_KIN).
// Chosen where the LDS of three waves per SIMD fits in 156 of the CU's 160
// KiB (a variant at 158 KiB, accepted by the occupancy query, ran 15%
// slower, as if a workgroup less fitted).  Against the two-wave form with
// the cache it measured 5% faster without the thermal phase and 9% with it
// at N = 2048 (FP32, W = 128), 0% and 6% at N = 4096 (FP32, W = 256), 6%
// and 15% at N = 2048 (FP64, W = 256); and 2% and 5% slower at N = 1024
// (FP32) with one wave per workgroup (whose transforms wait at no barrier),
// which keeps the two-wave form.  (With the paired table loads, the lead at
// N = 2048 grew to 22% and 18%.)
template <class R, int N, int W, int POT>
struct FusedForm {
    // FP32-bulk renormalises the unitary block of every step
    static constexpr bool kRenorm = std::is_same<R, float>::value;
    // block-scan and reduction scratch, work item and flag
    static constexpr size_t kSmallBytes = (W / 64) * (sizeof(cx<double>) + 14 * sizeof(double)) + 16;
    static constexpr int kWaves = W / 64;
    // exchange buffer of the transforms with one pad element in 16 (FP32:
    // see dst32)
    static constexpr size_t kBuf16 = kRenorm ? dst32_buf_bytes<N, W>()
                                             : sizeof(cx<R>) * (size_t)padded_len<N, 4>();
    // LDS of a lean workgroup: FP32 the exchange buffer (one pad element in
    // 16) and the damping factors, FP64 the exchange buffer with one pad
    // element in 8
    static constexpr size_t kLeanLds =
        (kRenorm ? kBuf16 + sizeof(R) * N : sizeof(cx<R>) * (size_t)padded_len<N, 3>()) +
        kSmallBytes;
    static constexpr bool kLean = POT == QT_POTENTIAL_MUNICH && N / W == (kRenorm ? 16 : 8) &&
                                  kWaves >= 2 && 12 % kWaves == 0 &&
                                  (size_t)(12 / kWaves) * kLeanLds <= 156u * 1024u;
    // LDS padding of the FP64 forms' transforms: one element in 8 (fewer
    // bank conflicts of their 16-byte exchanges than one in 16: 0.70 against
    // 1.19 conflict cycles per active LDS cycle at N = 2048, 2% faster); FP32
    // one in 16 (its LDS is at the limit)
    static constexpr int kPadS = kRenorm ? 4 : 3;
    // the damping factors between the half-steps in LDS (lean FP32)
    static constexpr bool kDmLds = kLean && kRenorm;
    // exchange buffer of the transforms
    static constexpr size_t kBufBytes = kRenorm ? dst32_buf_bytes<N, W>()
                                                : sizeof(cx<R>) * (size_t)padded_len<N, kPadS>();
    // per-lane cache of the phase factors C_m between the two half-steps of a
    // step, kept when it still leaves room for two workgroups per CU
    static constexpr bool kCache = !kLean && kBufBytes + sizeof(cx<R>) * N <= 80u * 1024u;
    static constexpr int kWavesPerEU = kLean ? 3 : 2;
};

template <class R, int N, int W, int POT>
__global__ __launch_bounds__(W) __attribute__((amdgpu_waves_per_eu(FusedForm<R, N, W, POT>::kWavesPerEU)))
void fused_kernel(FusedArgs A)
{
    using PL = Plan<N, W>;
    using FF = FusedForm<R, N, W, POT>;
    constexpr int R1 = PL::R1, T = PL::T;
    constexpr bool kRenorm = FF::kRenorm;
    constexpr bool kLean = FF::kLean;
    __shared__ __attribute__((aligned(16))) char buf[FF::kBufBytes];
    __shared__ cx<double> wsum[W / 64];
    __shared__ double red[14 * (W / 64)];
    __shared__ int s_item;
    __shared__ int s_zdone;
    constexpr bool kCache = FF::kCache;
    constexpr bool kStaticCache = kCache && W > 64;
    __shared__ cx<R> fac[kCache ? N : 1];
    // the lean FP32 form's damping factors between the half-steps
    __shared__ __attribute__((aligned(16))) R dms[FF::kDmLds ? N : 1];

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

        cx<R> a[R1], b[R1];
        // FP32-bulk: the state is scl times the stored values.  The norm
        // correction of a step is often below half an FP32 ulp, so that
        // multiplying the values by it would change none of them and its
        // sign, the same step after step, would add up; it is kept in FP64
        // instead (and in the checkpoint) and folded into the values when
        // it is large, at a jump and at the end.
        double scl = 1.0;
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
            scl = s.scl;
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
        // one potential per kernel: its own register allocation
        constexpr bool ksu = POT == QT_POTENTIAL_KSU;
        const cx<R>* ksu_tab = static_cast<const cx<R>*>(g.ksu_phi);
        const double ksu_rsb = 1.25 / 0.1973269804;
        const double ksu_vsb = -kKsuA / ksu_rsb + kKsuSigma * ksu_rsb;
        const R dr = R(g.dr);
        const double xmax = (double)(N - 1) * g.dr * (double)(N - 1) * g.dr;
        int cur = 0;
        scl = uniform(scl);
        // without the thermal phase the cache of C_m holds the static phase
        // row of (l, colour) from here and after every jump (workgroups of
        // several waves: with one wave, N = 1024, it measured 9% slower than
        // reading the row every step)
        const bool static_c = kStaticCache && !ksu && !has_gamma;
        if (static_c && status == QT_TRAJ_OK) fill_static_phase<R, N, W>(fac, phase_row<R, N>(g, l, c), ln);
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
            // (both precisions: the series only in range)
            const bool fast = fabs(-0.5 * g.dt * cc * kh * T3) * xmax <= 0.5 &&
                              fabs(-0.5 * g.dt * cc * g.gamma_hat * T3) * xmax <= 0.78;

            R dm[Plan<N, W>::P];
            double n_in = 0.0;
            // the KSU potential's factors are computed per point; its
            // per-step scalars are FP64
            double md = 0.0, cI = 0.0;
            if constexpr (ksu) ksu_medium(Tn, g.md_factor, &md, &cI);
            const HalfStepKSU<R> hk{ksu_tab, dr, R(0.5 * g.dt), R(md), R(cI),
                                    R((double)l * (double)(l + 1) / g.mass), R(ksu_vsb)};
            if constexpr (ksu) {
                n_in = first_half<R, N, W, HalfStepKSU<R>, kCache, kRenorm>(a, b, hk, ls, fac, dm);
            } else {
                with_factor_kind(has_gamma, fast, [&](auto G, auto F) QT_INL {
                    const HalfStep<R, G, F> h{row, dr, zr, zi};
                    n_in = first_half<R, N, W, HalfStep<R, G, F>, kCache, kRenorm, kStaticCache,
                                      FF::kDmLds>(a, b, h, ls, fac, dm, dms);
                });
            }
            if constexpr (kRenorm) {
                kin_block32<N, W, kLean>(a, b, ls, buf, wsum, A.tw,
                                         static_cast<const cx<double>*>(g.kin), (n & 1) != 0);
            } else {
                const Kin<double>* kin = static_cast<const Kin<double>*>(g.kin);
                cx<double> pw[Plan<N, W>::R1];
                load_prew<double, N, W>(pw, prew, ls);
                cx<double>* bd = reinterpret_cast<cx<double>*>(buf);
                const cx<double>* tw_n = opaque(tw);
                dst1<double, N, W, true, kLean, FF::kPadS>(a, b, pw, prew, ls, bd, wsum, tw_n, kin);
                dst1<double, N, W, false, false, FF::kPadS>(a, b, pw, prew, ls, bd, wsum, opaque(tw_n),
                                                            nullptr);
            }
            // x: sum |D u|^2 after the first half-step (the norm the unitary
            // block receives), sum |C u|^2 (what it returns), sum |D C u|^2
            double x[3] = {n_in, 0.0, 0.0};
            if constexpr (ksu) {
                second_half<R, N, W, HalfStepKSU<R>, kCache, kRenorm>(a, b, hk, ls, fac, dm, x[1], x[2]);
            } else {
                with_factor_kind(has_gamma, fast, [&](auto G, auto F) QT_INL {
                    const HalfStep<R, G, F> h{opaque(row), dr, zr, zi};
                    // the lean form derives the points' radii anew rather
                    // than keeping those of the first half-step
                    const Lanes<N, W> l2(kLean ? opaque_lane(threadIdx.x) : ls.t);
                    second_half<R, N, W, HalfStep<R, G, F>, kCache, kRenorm, FF::kDmLds,
                                kLean && !kRenorm>(a, b, h, l2, fac, dm, x[1], x[2], dms);
                });
            }
            if constexpr (kRenorm) {
                // the block C DST kin DST C is unitary: restore the norm it
                // received (D commutes with the scaling)
                block_sum_vec<W, 3>(x, red);
                scl = uniform(scl * sqrt(x[0] / x[1]));
                norm = g.dr * x[2] * scl * scl;
                if (fabs(scl - 1.0) > 0x1p-10) {
                    add_scaled<R, N, W>(a, b, R(scl - 1.0));
                    scl = 1.0;
                }
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
                log_jump(g.out, idx, n_jumps, n, l, c);
                // (radii derived here: no register holds them across steps)
                const Lanes<N, W> lj(opaque_lane(threadIdx.x));
                sfor<0, R1>([&](auto Rr) QT_INL {
                    a[Rr] = scale(a[Rr], R(lj.ja + Rr * T) * dr);
                    b[Rr] = scale(b[Rr], R(lj.jb + Rr * T) * dr);
                });
                const double s2 = g.dr * block_sum<W>(sum_abs2<R, N, W>(a, b), red);
                const R f = R(1.0 / sqrt(s2));
                sfor<0, R1>([&](auto Rr) QT_INL {
                    a[Rr] = scale(a[Rr], f);
                    b[Rr] = scale(b[Rr], f);
                });
                norm = g.dr * block_sum<W>(sum_abs2<R, N, W>(a, b), red);
                scl = 1.0;
                r = uniform(uniform01(e.w[2]));
                n_jumps += 1;
                l = uniform(l);
                c = uniform(c);
                if (l > g.l_tab) {
                    status = QT_TRAJ_LMAX;
                    break;
                }
                if (static_c) fill_static_phase<R, N, W>(fac, phase_row<R, N>(g, l, c), ls);
            }
        }
        const bool done = status != QT_TRAJ_OK || step >= g.n_steps;
        if (done && scl != 1.0) {
            add_scaled<R, N, W>(a, b, R(scl - 1.0));
            scl = 1.0;
        }
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
                s.scl = scl; s.pad2 = 0.0;
                g.st[idx] = s;
            }
        }
    }
}


template <class R, int N, int W, int POT>
hipError_t launch_fused(const FusedArgs& a, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((fused_kernel<R, N, W, POT>), dim3(grid), dim3(W), 0, s, a);
    return hipGetLastError();
}

template <class R, int N, int W, int POT>
int occupancy_fused()
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fused_kernel<R, N, W, POT>, W, 0) !=
        hipSuccess)
        return 0;
    return blocks;
}

struct FusedEntry {
    int prec, N, W;
    fused_launcher launch;
    int (*occ)();
};

}  // namespace qt
