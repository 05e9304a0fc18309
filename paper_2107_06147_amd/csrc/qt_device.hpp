// qt_device.hpp -- device building blocks of the quantum-trajectory kernels
// for gfx950 (CDNA4): complex arithmetic, the Philox4x64-10 counter RNG,
// in-register DFTs, LDS Stockham FFT passes, the symmetric DST-I wrapper and
// workgroup reductions.
//
// Layout of one trajectory's wave function inside a workgroup of W lanes
// (W a multiple of 64), N points, P = N/W complex values per lane:
//   R1 = P/2, T = 2W = N/R1.  Lane t holds two "mirror" columns
//     a[r] = u[ja + r T],  b[r] = u[jb + r T],  r = 0..R1-1,
//   with ja = t and jb = T - t (jb = W for lane 0).  The mirror point N - m of
//   every point m a lane holds is held by the same lane, which is what the
//   DST-I pre- and post-processing need.  This is also the input layout of
//   the first radix-R1 pass and the output layout of the last radix-R1 pass
//   of a Stockham FFT of length N.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

#include "qt_internal.h"
#include "qt_philox.h"

namespace qt {

// ---------------------------------------------------------------- basics --

// Lambdas handed to sfor must be inlined so that register arrays indexed by
// their compile-time index stay in registers.
#define QT_INL __attribute__((always_inline))

template <int B, int E, class F>
__device__ __forceinline__ void sfor(F&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        sfor<B + 1, E>(f);
    }
}

template <class R>
struct alignas(2 * sizeof(R)) cx {
    R re, im;
};

template <class R> __device__ __forceinline__ cx<R> mk(R a, R b) { cx<R> z; z.re = a; z.im = b; return z; }
template <class R> __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return mk(a.re + b.re, a.im + b.im); }
template <class R> __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return mk(a.re - b.re, a.im - b.im); }
template <class R> __device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b)
{
    return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <class R> __device__ __forceinline__ cx<R> scale(cx<R> a, R s) { return mk(a.re * s, a.im * s); }
// acc + |a|^2 in FP64 as two fused multiply-adds (the squares of FP32
// values are exact in FP64)
template <class R> __device__ __forceinline__ void add_abs2(double& acc, cx<R> a)
{
    const double x = (double)a.re, y = (double)a.im;
    acc = fma(y, y, fma(x, x, acc));
}

// Hides a pointer's value from the optimiser so that table loads through it
// stay inside the time loop instead of being hoisted into registers for the
// whole kernel (which would cost occupancy).
template <class T>
__device__ __forceinline__ const T* opaque(const T* p)
{
    // the pointer is wave-uniform: keep it in scalar registers
    const uint64_t u = reinterpret_cast<uint64_t>(p);
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    asm volatile("" : "+s"(lo), "+s"(hi));
    return reinterpret_cast<const T*>(((uint64_t)hi << 32) | lo);
}

// Loads of table element i through a global-address-space pointer with a
// 32-bit byte offset: the compiler then addresses them as scalar base +
// one vector register (no 64-bit address arithmetic per load, and no flat
// accesses that would also hold up the LDS wait counter).
#define QT_GLOBAL __attribute__((address_space(1)))
template <class R>
__device__ __forceinline__ cx<R> ldg(const cx<R>* p, uint32_t i)
{
    typedef R v2 __attribute__((ext_vector_type(2)));
    const v2 v = *(const QT_GLOBAL v2*)((const QT_GLOBAL char*)p + i * (uint32_t)sizeof(cx<R>));
    cx<R> z;
    z.re = v.x;
    z.im = v.y;
    return z;
}
// Two consecutive table elements i, i + 1 (i even: 16-byte aligned) in one load.
__device__ __forceinline__ void ldg_pair(const cx<float>* p, uint32_t i, cx<float>& x, cx<float>& y)
{
    typedef float v4 __attribute__((ext_vector_type(4)));
    const v4 v = *(const QT_GLOBAL v4*)((const QT_GLOBAL char*)p + i * (uint32_t)sizeof(cx<float>));
    x.re = v.x;
    x.im = v.y;
    y.re = v.z;
    y.im = v.w;
}
// Kinetic factor of one momentum (one complex value).
template <class R> struct Kin { cx<R> v; };
template <class R>
__device__ __forceinline__ Kin<R> ldg(const Kin<R>* p, uint32_t i)
{
    Kin<R> k;
    k.v = ldg(reinterpret_cast<const cx<R>*>(p), i);
    return k;
}
template <class R>
__device__ __forceinline__ R ldg(const R* p, uint32_t i)
{
    return *(const QT_GLOBAL R*)((const QT_GLOBAL char*)p + i * (uint32_t)sizeof(R));
}

// Same for the lane id: address arithmetic derived from it is then redone
// next to its use in every step instead of being kept live in registers
// across the whole time loop.
__device__ __forceinline__ int opaque_lane(int t)
{
    asm volatile("" : "+v"(t));
    return t;
}

// LDS index with one pad element every 2^S (spreads power-of-two strides
// over the banks); S = 4 unless a kernel asks for another.
template <int S = 4>
__device__ __forceinline__ int pad(int i) { return i + (i >> S); }
// pad(base + C) for a compile-time C, as a constant offset from pad(base).
// Valid when the low S bits of base and C do not carry into bit S, which
// holds for every access below for S = 3, 4 and 5: each one is base + C
// with base mod 2^S and C mod 2^S together below 2^S (all sizes, strides
// and radices are powers of two; the exchange writes pair j mod NS with
// multiples of NS, the sine transform's post-processing and prefix sum an
// even base with the odd offset 1, a multiple of 2 CH with offsets below
// 2 CH).  The offset then goes into the LDS instruction's immediate field.
template <int C, int S = 4> constexpr int padc() { return C + (C >> S); }
template <int N, int S = 4> constexpr int padded_len() { return N + (N >> S); }

// cos(2 pi k / 64), k = 0..63
constexpr double kCos64[64] = {
    1, 0.99518472667219693, 0.98078528040323043, 0.95694033573220882,
    0.92387953251128674, 0.88192126434835505, 0.83146961230254524, 0.77301045336273699,
    0.70710678118654757, 0.63439328416364549, 0.55557023301960229, 0.47139673682599781,
    0.38268343236508984, 0.29028467725446233, 0.19509032201612833, 0.09801714032956077,
    6.123233995736766e-17, -0.098017140329560645, -0.19509032201612819, -0.29028467725446216,
    -0.38268343236508973, -0.4713967368259977, -0.55557023301960196, -0.63439328416364538,
    -0.70710678118654746, -0.77301045336273699, -0.83146961230254535, -0.88192126434835494,
    -0.92387953251128674, -0.95694033573220882, -0.98078528040323043, -0.99518472667219682,
    -1, -0.99518472667219693, -0.98078528040323043, -0.95694033573220894,
    -0.92387953251128685, -0.88192126434835505, -0.83146961230254546, -0.7730104533627371,
    -0.70710678118654768, -0.63439328416364593, -0.55557023301960218, -0.47139673682599786,
    -0.38268343236509034, -0.29028467725446244, -0.19509032201612866, -0.098017140329560451,
    -1.8369701987210297e-16, 0.09801714032956009, 0.1950903220161283, 0.29028467725446205,
    0.38268343236509, 0.47139673682599759, 0.55557023301960184, 0.6343932841636456,
    0.70710678118654735, 0.77301045336273666, 0.83146961230254524, 0.88192126434835483,
    0.92387953251128652, 0.95694033573220882, 0.98078528040323032, 0.99518472667219693,
};

// d * exp(-2 pi i k / M), with k, M compile-time constants (M <= 64)
template <int M, int K, class R>
__device__ __forceinline__ cx<R> twiddle_mul(cx<R> d)
{
    constexpr int k = K % M;
    if constexpr (k == 0) {
        return d;
    } else if constexpr (4 * k == M) {          // -i
        return mk(d.im, -d.re);
    } else if constexpr (2 * k == M) {          // -1
        return mk(-d.re, -d.im);
    } else if constexpr (4 * k == 3 * M) {      // +i
        return mk(-d.im, d.re);
    } else if constexpr (8 * k == M) {          // (1 - i)/sqrt2
        constexpr R c = R(0.70710678118654752440);
        return mk((d.re + d.im) * c, (d.im - d.re) * c);
    } else if constexpr (8 * k == 3 * M) {      // (-1 - i)/sqrt2
        constexpr R c = R(0.70710678118654752440);
        return mk((d.im - d.re) * c, -(d.re + d.im) * c);
    } else {
        constexpr int idx = (k * 64 / M) % 64;
        constexpr R c = R(kCos64[idx]);
        constexpr R s = R(kCos64[(idx + 48) % 64]);   // sin(2 pi k/M)
        // (re + i im)(c - i s)
        return mk(d.re * c + d.im * s, d.im * c - d.re * s);
    }
}

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }
constexpr int bitrev(int i, int bits)
{
    int r = 0;
    for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
    return r;
}

// In-register forward DFT of length RAD (power of two <= 64):
// v[k] <- sum_j v[j] exp(-2 pi i j k / RAD).  Radix-2 decimation in
// frequency; the bit-reversed output order is undone by register renaming.
template <int RAD, class R>
__device__ __forceinline__ void dft(cx<R>* v)
{
    if constexpr (RAD == 1) {
        return;
    } else {
        sfor<0, ilog2(RAD)>([&](auto S) QT_INL {
            constexpr int half = RAD >> (S + 1);
            sfor<0, RAD / (2 * half)>([&](auto G) QT_INL {
                constexpr int s0 = G * 2 * half;
                sfor<0, half>([&](auto K) QT_INL {
                    constexpr int k = K;
                    cx<R> a = v[s0 + k], b = v[s0 + k + half];
                    v[s0 + k] = a + b;
                    v[s0 + k + half] = twiddle_mul<2 * half, k>(a - b);
                });
            });
        });
        cx<R> t[RAD];
        sfor<0, RAD>([&](auto I) QT_INL { t[bitrev(I, ilog2(RAD))] = v[I]; });
        sfor<0, RAD>([&](auto I) QT_INL { v[I] = t[I]; });
    }
}

// ------------------------------------------------------------ FFT plan ----

// Radix plan of a length-N FFT on W lanes: the first and the last pass have
// radix R1 = P/2 with two (mirror) butterflies per lane; the middle passes
// split M = N / R1^2 as evenly as possible into powers of two <= P.
template <int N, int W>
struct Plan {
    static constexpr int P = N / W;
    static constexpr int R1 = P / 2;
    static constexpr int T = 2 * W;
    static constexpr int MID = N / (R1 * R1);
    static constexpr int LOGP = ilog2(P);
    static constexpr int LOGMID = ilog2(MID);
    static constexpr int NMID = LOGMID == 0 ? 0 : (LOGMID + LOGP - 1) / LOGP;
    static constexpr int NPASS = 2 + NMID;
    static constexpr int mid_log(int i)
    {
        // split LOGMID into NMID parts, larger parts first
        return LOGMID / NMID + (i < LOGMID % NMID ? 1 : 0);
    }
    static constexpr int radix(int p)
    {
        return (p == 0 || p == NPASS - 1) ? R1 : (1 << mid_log(p - 1));
    }
    static constexpr int ns(int p)
    {
        int s = 1;
        for (int q = 0; q < p; ++q) s *= radix(q);
        return s;
    }
    static_assert(W % 64 == 0, "whole wavefronts");
    static_assert(P >= 4 && (P & (P - 1)) == 0, "P = N/W must be a power of two >= 4");
};

template <int N, int W>
struct Lanes {
    int t, ja, jb;
    __device__ __forceinline__ explicit Lanes(int tid)
    {
        t = tid;
        ja = tid;
        jb = tid == 0 ? W : 2 * W - tid;
    }
};

// Twiddle factors of pass p for this lane's butterflies (none for the first
// pass, whose stride is 1): w^{r k}, r = 1..RAD-1, for butterfly k, w =
// exp(-2 pi i / L), L = NS RAD.  FP32 reads each from a level table
// (load_level; its rounding is what limits the FP32 form's accuracy).  FP64
// reads w^k only, from the natural table of length N at k N/L (load), and
// forms the other powers as products of two lower ones, w^{r k} = w^{h k}
// w^{(r-h) k} with h the largest power of two below r (r/2 for a power of
// two): at most three products deep, a few units of the FP64 roundoff, and
// one table read where there were RAD - 1 (table reads, not arithmetic, are
// what the transforms wait for).
template <class R, int N, int W, int p>
struct PassTwiddles {
    using PL = Plan<N, W>;
    static constexpr int RAD = PL::radix(p);
    static constexpr int NS = PL::ns(p);
    static constexpr int B = PL::P / RAD;
    static constexpr int K = NS > 1 ? B * (RAD - 1) : 1;
    cx<R> w[K];
    __device__ __forceinline__ static int bfly(const Lanes<N, W>& ln, int q)
    {
        constexpr bool edge = (p == 0 || p == PL::NPASS - 1);
        return edge ? (q == 0 ? ln.ja : ln.jb) : q * W + ln.t;
    }
    __device__ __forceinline__ void load(const Lanes<N, W>& ln, const cx<R>* tw)
    {
        static_assert(sizeof(R) == sizeof(double), "FP32 twiddles come from level tables");
        if constexpr (NS > 1) {
            sfor<0, B>([&](auto Q) QT_INL {
                const int k = bfly(ln, Q) & (NS - 1);
                cx<R>* wq = w + Q * (RAD - 1);   // wq[r - 1] = w^{r k}
                wq[0] = ldg(tw, k * (N / (NS * RAD)));
                sfor<2, RAD>([&](auto Rr) QT_INL {
                    constexpr int r = Rr;
                    constexpr int h = (r & (r - 1)) ? (1 << ilog2(r)) : r / 2;
                    wq[r - 1] = wq[h - 1] * wq[r - h - 1];
                });
            });
        }
    }
    // The same from a level table: level L = NS RAD (4, 8, ..., N) holds
    // w_L^{r k} = exp(-2 pi i r k / L) at entry level_index(L, r, k) (r =
    // 1..7, k < L/2): the powers r = 1, 2 (3, 4 and 5, 6) of one k side by
    // side, one 16-byte load, the pairs of consecutive k consecutive, so that
    // the lanes of a pass read consecutive entries (the natural table at r k
    // N/L spreads them over up to 8 r times as many cache lines) with half
    // the load instructions of one per power.
    __device__ __forceinline__ void load_level(const Lanes<N, W>& ln, const cx<R>* lev)
    {
        static_assert(RAD <= 8, "the level tables hold the powers r <= 7");
        if constexpr (NS > 1) {
            constexpr int L = NS * RAD;
            sfor<0, B>([&](auto Q) QT_INL {
                const int k = bfly(ln, Q) & (NS - 1);
                cx<R>* wq = w + Q * (RAD - 1);
                sfor<1, RAD>([&](auto Rr) QT_INL {
                    constexpr int r = Rr;
                    if constexpr (r % 2 == 1) {
                        if constexpr (r + 1 < RAD)
                            ldg_pair(lev, (uint32_t)level_index(L, r, k), wq[r - 1], wq[r]);
                        else
                            wq[r - 1] = ldg(lev, (uint32_t)level_index(L, r, k));
                    }
                });
            });
        }
    }
};

// Butterflies of pass p: twiddle (passes after the first), then the DFT of
// each of this lane's B groups of RAD values.
template <class R, int N, int W, int p>
__device__ __forceinline__ void fft_pass(cx<R>* v, const PassTwiddles<R, N, W, p>& cur)
{
    using TW = PassTwiddles<R, N, W, p>;
    constexpr int RAD = TW::RAD;
    sfor<0, TW::B>([&](auto Q) QT_INL {
        constexpr int q = Q;
        if constexpr (TW::NS > 1) {
            sfor<1, RAD>([&](auto Rr) QT_INL {
                constexpr int r = Rr;
                v[q * RAD + r] = v[q * RAD + r] * cur.w[q * (RAD - 1) + r - 1];
            });
        }
        dft<RAD>(v + q * RAD);
    });
}

// The exchange after pass p through LDS into the input layout of pass p + 1:
// write, barrier, read.  Butterfly j of a pass with stride NS reads
// x[j + r N/RAD] and writes y[(j/NS) NS RAD + j%NS + r NS].
template <class R, int N, int W, int p, int S = 4>
__device__ __forceinline__ void fft_exchange(cx<R>* v, const Lanes<N, W>& ln, cx<R>* buf)
{
    using PL = Plan<N, W>;
    using TW = PassTwiddles<R, N, W, p>;
    constexpr int RAD = TW::RAD;
    constexpr int NS = TW::NS;
    sfor<0, TW::B>([&](auto Q) QT_INL {
        constexpr int q = Q;
        const int j = TW::bfly(ln, q);
        cx<R>* dst = buf + pad<S>((j / NS) * NS * RAD + (j & (NS - 1)));
        sfor<0, RAD>([&](auto Rr) QT_INL { dst[padc<Rr * NS, S>()] = v[q * RAD + Rr]; });
    });
    __syncthreads();
    constexpr int RAD2 = PL::radix(p + 1);
    constexpr int B2 = PL::P / RAD2;
    sfor<0, B2>([&](auto Q) QT_INL {
        constexpr int q = Q;
        const int j = PassTwiddles<R, N, W, p + 1>::bfly(ln, q);
        const cx<R>* src = buf + pad<S>(j);
        sfor<0, RAD2>([&](auto Rr) QT_INL { v[q * RAD2 + Rr] = src[padc<Rr * (N / RAD2), S>()]; });
    });
}

// The passes p.. of the FFT.  The next pass's twiddles are loaded before
// the exchange, so that their latency overlaps it; a barrier follows each
// exchange's read, so that the next exchange may overwrite the buffer.
template <class R, int N, int W, int p, int S = 4>
__device__ __forceinline__ void fft_passes(cx<R>* v, const Lanes<N, W>& ln, cx<R>* buf,
                                           const cx<R>* __restrict__ tw,
                                           const PassTwiddles<R, N, W, p>& cur)
{
    fft_pass<R, N, W, p>(v, cur);
    if constexpr (p + 1 < Plan<N, W>::NPASS) {
        PassTwiddles<R, N, W, p + 1> nxt;
        nxt.load(ln, opaque(tw));
        fft_exchange<R, N, W, p, S>(v, ln, buf);
        __syncthreads();
        fft_passes<R, N, W, p + 1, S>(v, ln, buf, tw, nxt);
    }
}

// The twiddles of every pass from p on, for FFTs that run more than once
// with the same table and lanes.
template <class R, int N, int W, int p, bool END = (p >= Plan<N, W>::NPASS)>
struct AllTwiddles {
    PassTwiddles<R, N, W, p> cur;
    AllTwiddles<R, N, W, p + 1> rest;
    __device__ __forceinline__ void load_level(const Lanes<N, W>& ln, const cx<R>* lev)
    {
        cur.load_level(ln, lev);
        rest.load_level(ln, lev);
    }
};
template <class R, int N, int W, int p>
struct AllTwiddles<R, N, W, p, true> {
    __device__ __forceinline__ void load_level(const Lanes<N, W>&, const cx<R>*) {}
};

// fft_passes with the twiddles already in registers, and two exchange
// buffers: exchanges alternate between buf and buf2, with no barrier after
// the read (a wave writes a buffer again only after the barrier of the
// exchange in between, which every wave reaches after its reads of that
// buffer).  The caller owes a barrier before it next writes the buffer of
// the last exchange, or the other one before that.
template <class R, int N, int W, int p>
__device__ __forceinline__ void fft_passes_held(cx<R>* v, const Lanes<N, W>& ln, cx<R>* buf,
                                                cx<R>* buf2, const AllTwiddles<R, N, W, p>& tws)
{
    fft_pass<R, N, W, p>(v, tws.cur);
    if constexpr (p + 1 < Plan<N, W>::NPASS) {
        fft_exchange<R, N, W, p>(v, ln, buf);
        fft_passes_held<R, N, W, p + 1>(v, ln, buf2, buf, tws.rest);
    }
}

// fft_passes_held with two exchange buffers as there, but each pass's
// twiddles loaded (from a level table) before the exchange that precedes it
// instead of held for the whole FFT (fewer registers; their latency
// overlaps the exchange).
template <class R, int N, int W, int p>
__device__ __forceinline__ void fft_passes_db(cx<R>* v, const Lanes<N, W>& ln, cx<R>* buf,
                                              cx<R>* buf2, const cx<R>* __restrict__ lev,
                                              const PassTwiddles<R, N, W, p>& cur)
{
    fft_pass<R, N, W, p>(v, cur);
    if constexpr (p + 1 < Plan<N, W>::NPASS) {
        PassTwiddles<R, N, W, p + 1> nxt;
        nxt.load_level(ln, opaque(lev));
        fft_exchange<R, N, W, p>(v, ln, buf);
        fft_passes_db<R, N, W, p + 1>(v, ln, buf2, buf, lev, nxt);
    }
}

// The values of this lane's slots (slot r < R1: point ja + rT, slot R1 + r:
// jb + rT) from an FP32 table of length N in mirror pairs: entry e < N/2 (16
// bytes) holds the values at e and N - e (at 0 and N/2 for e = 0).  Every
// lane t > 0 reads the pairs (t + rT, with its slot b[R1-1-r]) and (T - t +
// rT, with a[R1-1-r]), r < R1/2, at consecutive entries with its
// neighbours: half the loads of one per point, each as coalesced.  Lane 0
// (points rT and W + rT) finds the partners of its upper slots in the other
// entry of the two, selected per lane.
template <int N, int W>
__device__ __forceinline__ void load_mirror_pairs(const cx<float>* tab, const Lanes<N, W>& ln,
                                                  cx<float>* v)
{
    constexpr int R1 = Plan<N, W>::R1, T = Plan<N, W>::T, Q = R1 / 2;
    const bool lane0 = ln.t == 0;
    cx<float> ax[Q], ay[Q], bx[Q], by[Q];
    sfor<0, Q>([&](auto Rr) QT_INL {
        ldg_pair(tab, 2u * (uint32_t)(ln.ja + Rr * T), ax[Rr], ay[Rr]);
        ldg_pair(tab, 2u * (uint32_t)(ln.jb + Rr * T), bx[Rr], by[Rr]);
    });
    sfor<0, Q>([&](auto Rr) QT_INL {
        constexpr int r = Rr;
        v[r] = ax[r];
        v[R1 + r] = bx[r];
        v[R1 - 1 - r] = lane0 ? ay[(r + 1) % Q] : by[r];
        v[2 * R1 - 1 - r] = lane0 ? by[r] : ay[r];
    });
}
// ------------------------------------------------------- reductions -------

// Cross-lane moves with the data-parallel-primitives (DPP) modifier: a VALU
// move that reads another lane of the same row of 16 (or, for the two
// broadcasts, the last lane of the previous row / of row 1), no LDS round
// trip.  Lanes without a source, and rows left out by ROWS, read 0.
enum : int {
    kDppSwap1 = 0xB1,          // quad_perm [1,0,3,2]
    kDppSwap2 = 0x4E,          // quad_perm [2,3,0,1]
    kDppRowShr1 = 0x111,       // row_shr:n = 0x110 + n
    kDppRowMirror = 0x140,
    kDppRowHalfMirror = 0x141,
    kDppBcast15 = 0x142,       // lane 15 of each row to the next row
    kDppBcast31 = 0x143,       // lane 31 to rows 2 and 3
};
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ float dpp(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL,
                                                                 ROWS, 0xF, true));
}
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp(double x)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROWS, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROWS, 0xF, true);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Sum over the 64 lanes of the wave, as a wave-uniform value.
__device__ __forceinline__ double wave_sum(double x)
{
    x += dpp<kDppSwap1>(x);
    x += dpp<kDppSwap2>(x);
    x += dpp<kDppRowHalfMirror>(x);
    x += dpp<kDppRowMirror>(x);          // every lane: its row's sum
    x += dpp<kDppBcast15, 0xA>(x);       // rows 1, 3: rows 0+1, 2+3
    x += dpp<kDppBcast31, 0xC>(x);       // row 3: all rows
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, 63);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), 63);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Inclusive prefix sum over the 64 lanes of the wave (lane order).
template <class T>
__device__ __forceinline__ T wave_inclusive_scan(T x)
{
    x += dpp<kDppRowShr1>(x);
    x += dpp<kDppRowShr1 + 1>(x);
    x += dpp<kDppRowShr1 + 3>(x);
    x += dpp<kDppRowShr1 + 7>(x);        // scan within each row of 16
    x += dpp<kDppBcast15, 0xA>(x);       // rows 1, 3 add the end of rows 0, 2
    x += dpp<kDppBcast31, 0xC>(x);       // rows 2, 3 add the end of row 1
    return x;
}

// The value of lane 0 as a wave-uniform value (scalar register): lets the
// compiler treat data that is identical on every lane (block reductions,
// per-trajectory scalars) as uniform, so branches on it stay scalar.
__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ double uniform(double x)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ int64_t uniform(int64_t x)
{
    const uint64_t u = (uint64_t)x;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Sum over the workgroup; every lane gets the total.  `red` holds W/64
// doubles of LDS.
template <int W>
__device__ __forceinline__ double block_sum(double x, double* red)
{
    x = wave_sum(x);
    if constexpr (W > 64) {
        const int wave = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) red[wave] = x;
        __syncthreads();
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < W / 64; ++w) s += red[w];
        __syncthreads();
        return uniform(s);
    } else {
        return uniform(x);
    }
}

// Exclusive prefix sum over the lanes of the workgroup (lane order).
template <int W, class R>
__device__ __forceinline__ cx<R> block_exclusive_scan(cx<R> x, cx<R>* wsum)
{
    cx<R> inc = mk(wave_inclusive_scan(x.re), wave_inclusive_scan(x.im));
    cx<R> exc = inc - x;
    if constexpr (W > 64) {
        const int wave = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 63) wsum[wave] = inc;
        __syncthreads();
        cx<R> off = mk(R(0), R(0));
        for (int w = 0; w < wave; ++w) off = off + wsum[w];
        exc = exc + off;
    }
    return exc;
}

// Pre-processing weights of the points a[r] of the mirror layout (see
// dst1): pw[r] = (p, q) at m = ja + r T.  The same for both transforms of a
// step.
template <class R, int N, int W>
__device__ __forceinline__ void load_prew(cx<R>* pw, const cx<R>* prew, const Lanes<N, W>& ln)
{
    constexpr int R1 = Plan<N, W>::R1, T = Plan<N, W>::T;
    prew = opaque(prew);
    sfor<0, R1>([&](auto Rr) QT_INL { pw[Rr] = ldg(prew, ln.ja + Rr * T); });
}

// ------------------------------------------------------------- DST-I ------
//
// F_k = sum_{m=1}^{N-1} x_m sin(pi m k / N) on complex data with one complex
// FFT of length N (the sine transform is real, so it acts on re and im
// alike).  With s_m = sin(pi m/N):
//   y_m = s_m (x_m + x_{N-m}) + (x_m - x_{N-m})/2,   Y = FFT_N(y),
//   F_{2k}   = (i/2) (Y_k - Y_{N-k}),
//   D_k      = (Y_k + Y_{N-k})/2 = F_{2k+1} - F_{2k-1},
//   F_{2k+1} = sum_{q=0}^{k} D_q - Y_0/2.
// The pre-processing is done on the pair (m, N-m) at once and computes y/2:
//   y_m/2 = p_m x_m + q_m x_{N-m},  y_{N-m}/2 = p_m x_{N-m} + q_m x_m,
// p = (s + 1/2)/2, q = (s - 1/2)/2 (s_{N-m} = s_m); the halving cancels the
// factors 1/2 of the post-processing.
// On entry a/b hold x in the mirror layout and pw the weights (load_prew);
// prew is the weight table (lane 0 reads its second column from it).  On
// exit a/b hold F (times the kinetic factor of each output if KIN) in the
// same layout.  The kinetic factors are loaded before the prefix sum, whose
// exchanges hide their latency, or, LATE_KIN, where they are used (fewer
// registers held across the sum).
template <class R, int N, int W, bool KIN, bool LATE_KIN = false, int S = 4>
__device__ __forceinline__ void dst1(cx<R>* a, cx<R>* b, const cx<R>* pw, const cx<R>* prew,
                                     const Lanes<N, W>& ln_in, cx<R>* buf, cx<R>* wsum,
                                     const cx<R>* __restrict__ tw,
                                     const Kin<R>* __restrict__ kin)
{
    using PL = Plan<N, W>;
    constexpr int R1 = PL::R1;
    constexpr int T = PL::T;
    const Lanes<N, W> ln(opaque_lane(ln_in.t));
    const bool lane0 = ln.t == 0;
    cx<R> v[PL::P];
    auto mix = [](cx<R> x, cx<R> y, cx<R> w) QT_INL {
        return mk(w.re * x.re + w.im * y.re, w.re * x.im + w.im * y.im);
    };
    // pre-processing.  Every lane but 0: the mirror of a[r] (m = t + r T) is
    // b[R1-1-r] (N - m = T - t + (R1-1-r) T).
    sfor<0, R1>([&](auto Rr) QT_INL {
        constexpr int r = Rr;
        const cx<R> x = a[r], y = b[R1 - 1 - r];
        v[r] = mix(x, y, pw[r]);
        v[2 * R1 - 1 - r] = mix(y, x, pw[r]);
    });
    if (lane0) {
        // lane 0 holds m = r T (mirror (R1 - r) T, itself for r = 0 and
        // R1/2) and m = W + r T (mirror W + (R1-1-r) T): redone here, by
        // the first wave only
        sfor<0, R1 / 2 + 1>([&](auto Rr) QT_INL {
            constexpr int r = Rr;
            constexpr int rm = (R1 - r) % R1;
            const cx<R> x = a[r], y = a[rm];
            v[r] = mix(x, y, pw[r]);
            if constexpr (rm != r) v[rm] = mix(y, x, pw[r]);
        });
        const cx<R>* tab = opaque(prew);
        sfor<0, R1 / 2>([&](auto Rr) QT_INL {
            constexpr int r = Rr;
            const cx<R> w = ldg(tab, W + r * T);
            const cx<R> x = b[r], y = b[R1 - 1 - r];
            v[R1 + r] = mix(x, y, w);
            v[2 * R1 - 1 - r] = mix(y, x, w);
        });
    }
    {
        PassTwiddles<R, N, W, 0> none;
        fft_passes<R, N, W, 0, S>(v, ln, buf, tw, none);
    }
    // post-processing: pairs (k, N-k), even outputs F_{2k} and differences
    // D_k for k < N/2 (Y here is half the FFT of y)
    auto mul_i = [](cx<R> z) QT_INL { return mk(-z.im, z.re); };
    sfor<0, R1 / 2>([&](auto Rr) QT_INL {
        constexpr int r = Rr;
        {   // k = ja + r T, N - k = jb + (R1-1-r) T
            const cx<R> y = v[r], yp = v[2 * R1 - 1 - r];
            cx<R>* dst = buf + pad<S>(2 * ln.ja);
            dst[padc<2 * r * T, S>()] = mul_i(y - yp);
            dst[padc<2 * r * T, S>() + 1] = y + yp;
        }
        {   // k = jb + r T, N - k = ja + (R1-1-r) T
            const cx<R> y = v[R1 + r], yp = v[R1 - 1 - r];
            cx<R>* dst = buf + pad<S>(2 * ln.jb);
            dst[padc<2 * r * T, S>()] = mul_i(y - yp);
            dst[padc<2 * r * T, S>() + 1] = y + yp;
        }
    });
    if (lane0) {
        // lane 0: N - r T = (R1 - r) T and N - (W + r T) = W + (R1-1-r) T;
        // rewrites its entries
        sfor<0, R1 / 2>([&](auto Rr) QT_INL {
            constexpr int r = Rr;
            {
                const cx<R> y = v[r], yp = v[(R1 - r) % R1];
                cx<R>* dst = buf + pad<S>(2 * ln.ja);
                dst[padc<2 * r * T, S>()] = mul_i(y - yp);
                dst[padc<2 * r * T, S>() + 1] = y + yp;
            }
            {
                const cx<R> y = v[R1 + r], yp = v[2 * R1 - 1 - r];
                cx<R>* dst = buf + pad<S>(2 * ln.jb);
                dst[padc<2 * r * T, S>()] = mul_i(y - yp);
                dst[padc<2 * r * T, S>() + 1] = y + yp;
            }
        });
    }
    // kinetic factors of the outputs this lane ends up holding (mirror
    // layout), loaded here so that the exchanges below hide their latency
    constexpr bool kEarly = KIN && !LATE_KIN;
    Kin<R> kk[kEarly ? PL::P : 1];
    if constexpr (kEarly) {
        kin = opaque(kin);
        sfor<0, R1>([&](auto Rr) QT_INL {
            kk[Rr] = ldg(kin, ln.ja + Rr * T);
            kk[R1 + Rr] = ldg(kin, ln.jb + Rr * T);
        });
    }
    __syncthreads();
    // prefix sum of D_k over k = 0..N/2-1: contiguous chunks per lane
    constexpr int CH = N / (2 * W);
    const cx<R> d0 = buf[pad<S>(1)];
    cx<R> pre[CH];
    cx<R> run = mk(R(0), R(0));
    cx<R>* chunk = buf + pad<S>(2 * CH * ln.t);
    sfor<0, CH>([&](auto I) QT_INL {
        run = run + chunk[padc<2 * I + 1, S>()];
        pre[I] = run;
    });
    const cx<R> off = block_exclusive_scan<W>(run, wsum) - scale(d0, R(0.5));
    sfor<0, CH>([&](auto I) QT_INL { chunk[padc<2 * I + 1, S>()] = pre[I] + off; });
    __syncthreads();
    auto kmul = [&](cx<R> F, const Kin<R>& k) QT_INL { return F * k.v; };
    {
        const cx<R>* sa = buf + pad<S>(ln.ja);
        const cx<R>* sb = buf + pad<S>(ln.jb);
        const Kin<R>* kl = LATE_KIN ? opaque(kin) : kin;
        sfor<0, R1>([&](auto Rr) QT_INL {
            a[Rr] = sa[padc<Rr * T, S>()];
            b[Rr] = sb[padc<Rr * T, S>()];
            if constexpr (kEarly) {
                a[Rr] = kmul(a[Rr], kk[Rr]);
                b[Rr] = kmul(b[Rr], kk[R1 + Rr]);
            } else if constexpr (KIN) {
                a[Rr] = kmul(a[Rr], ldg(kl, ln.ja + Rr * T));
                b[Rr] = kmul(b[Rr], ldg(kl, ln.jb + Rr * T));
            }
        });
    }
    __syncthreads();
}

// --------------------------------------------------------- temperature ----

// Linear interpolation in the table; `cur` is a cursor that only moves
// forward (t grows with the step index).
__device__ __forceinline__ double temperature_at(const double* __restrict__ tau,
                                                 const double* __restrict__ Tt, int n, double t,
                                                 int& cur)
{
    if (t <= tau[0]) return Tt[0];
    if (t >= tau[n - 1]) return Tt[n - 1];
    while (!(tau[cur + 1] > t)) ++cur;
    const double w = (t - tau[cur]) / (tau[cur + 1] - tau[cur]);
    return Tt[cur] + (Tt[cur + 1] - Tt[cur]) * w;
}

}  // namespace qt
