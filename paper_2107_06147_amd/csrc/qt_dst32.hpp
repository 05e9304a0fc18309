// qt_dst32.hpp -- the sine transform of the FP32-bulk form.
//
// The DST-I of qt_device.hpp (dst1) takes one complex FFT of length N and
// recovers the odd outputs as a running sum of differences.  That sum
// integrates the rounding error of every earlier output: in FP32 the error
// of one transform grows like sqrt(N) times the unit roundoff, and a step
// repeats nearly the same error, so it builds up linearly over the steps
// (about 1e-3 relative after 1e3 steps at N = 2048).  The FP32 form
// therefore splits the transform once, along the pairs (m, N - m):
//   F_{2q}   = sum_{m<N/2} (x_m - x_{N-m}) sin(2 pi m q / N)
//            = DST-I of length M = N/2 of a-_m = x_m - x_{N-m},
//   F_{2q+1} = sum_{m<=M} (x_m + x_{N-m}) sin(pi m (2q+1) / N)   (x_{N/2} once)
//            = (-1)^q DCT-III_q of c_j = a+_{M-j},
// and takes the odd half with a well-conditioned length-M FFT in FP32 (the
// cosine transform of complex data via one FFT: every output a two-term
// sum with unit twiddles), the even half with dst1 of length M in FP64 (its
// running sum then carries FP64 rounding only).  The FFT work is that of
// one length-N FFT, a third of it in FP64 (same VALU rate as unpacked
// FP32).  Plans with four values per lane have no half-length plan; they
// widen the data and take dst1 of length N in FP64.
//
// Cosine transform (complex c_0..c_{M-1}, c_M = 0, theta = pi/(2M)):
//   V_0 = 2 c_0,  V_j = e^{i theta j} (c_j - i c_{M-j}),
//   v_n = sum_j V_j e^{2 pi i j n / M} = 2 X_{2n}            (n < M/2)
//                                     = 2 X_{2(M-1-n)+1}    (n >= M/2),
// X_q = sum_j c_j cos(theta j (2q+1)).  With c_j = a+_{M-j}:
//   F_{4n+1} = v_n / 2 (n < M/2),  F_{2N-4n-1} = -v_n / 2 (n >= M/2).
// The inverse DFT is conj(FFT(conj V)).
//
// Tables (one block, see ensure_tables): FP32 [FFT twiddles of length M |
// e^{-i pi j/N}, j < M], then FP64 [FFT twiddles of length M | DST-I weights
// of length M | FFT twiddles of length N | DST-I weights of length N].
// Kinetic factors in output order (cx<double>): entry n < M the factor of
// the odd output in slot n with its sign and 1/2, entry M + q that of F_{2q}.
#pragma once
#include "qt_device.hpp"

namespace qt {

template <int N>
struct Dst32Tables {
    static constexpr int M = N / 2;
    const cx<float>* tw32;     // FFT twiddles, length M
    const cx<float>* wd;       // e^{-i pi j / N}, j < M
    const cx<double>* tw64h;   // FFT twiddles, length M
    const cx<double>* pre64h;  // DST-I weights, length M
    const cx<double>* tw64;    // FFT twiddles, length N
    const cx<double>* pre64;   // DST-I weights, length N
    __device__ __forceinline__ explicit Dst32Tables(const void* base)
    {
        const char* p = static_cast<const char*>(base);
        tw32 = reinterpret_cast<const cx<float>*>(p);
        wd = tw32 + M;
        tw64h = reinterpret_cast<const cx<double>*>(p + 2 * (size_t)M * sizeof(cx<float>));
        pre64h = tw64h + M;
        tw64 = pre64h + M;
        pre64 = tw64 + N;
    }
};

__device__ __forceinline__ cx<double> widen(cx<float> z) { return mk((double)z.re, (double)z.im); }
__device__ __forceinline__ cx<float> narrow(cx<double> z) { return mk((float)z.re, (float)z.im); }
__device__ __forceinline__ cx<float> conjf(cx<float> z) { return mk(z.re, -z.im); }
// (p + i q) conjugated termwise: conj(p) + i conj(q)
__device__ __forceinline__ cx<float> conj_plus_iconj(cx<float> p, cx<float> q)
{
    return mk(p.re + q.im, q.re - p.im);
}
// FP32 value times an FP64 factor, rounded once
__device__ __forceinline__ cx<float> mulk(cx<float> f, cx<double> k)
{
    const double re = (double)f.re, im = (double)f.im;
    return mk((float)(re * k.re - im * k.im), (float)(re * k.im + im * k.re));
}

// LDS bytes of the exchange buffer (and of the block-scan scratch) that the
// FP32 transform of length N on W lanes needs.
template <int N, int W>
constexpr size_t dst32_buf_bytes()
{
    return Plan<N, W>::P >= 8 ? sizeof(cx<double>) * (size_t)padded_len<N / 2>()
                              : sizeof(cx<double>) * (size_t)padded_len<N>();
}

// On entry a/b hold x in the mirror layout of length N; on exit F (times the
// kinetic factor of each output if KIN) in the same layout.  buf: LDS of
// dst32_buf_bytes<N, W>(); wsum: W/64 cx<double> of LDS.
template <int N, int W, bool KIN>
__device__ __forceinline__ void dst32(cx<float>* a, cx<float>* b, const Lanes<N, W>& ln_in,
                                      void* buf, cx<double>* wsum, const void* tables,
                                      const cx<double>* __restrict__ kin)
{
    using PL = Plan<N, W>;
    constexpr int R1 = PL::R1, T = PL::T;
    const Dst32Tables<N> tb(opaque(static_cast<const char*>(tables)));
    if constexpr (PL::P < 8) {
        // widened: dst1 of length N in FP64
        const Lanes<N, W> ln(opaque_lane(ln_in.t));
        cx<double> A[R1], B[R1], pw[R1];
        sfor<0, R1>([&](auto Rr) QT_INL {
            A[Rr] = widen(a[Rr]);
            B[Rr] = widen(b[Rr]);
        });
        load_prew<double, N, W>(pw, tb.pre64, ln);
        dst1<double, N, W, false>(A, B, pw, tb.pre64, ln, static_cast<cx<double>*>(buf), wsum,
                                  tb.tw64, nullptr);
        // output k's factor in output order: even k at M + k/2, odd k at the
        // slot n of the half-length cosine transform (with its sign and 1/2)
        auto kfac = [&](int k) QT_INL {
            constexpr int M = N / 2;
            if (!KIN) return mk(1.0, 0.0);
            if ((k & 1) == 0) return ldg(kin, (uint32_t)(M + k / 2));
            const bool lo = ((k - 1) & 3) == 0;
            const int n = lo ? (k - 1) / 4 : (2 * N - 1 - k) / 4;
            const cx<double> f = ldg(kin, (uint32_t)n);
            return lo ? mk(2.0 * f.re, 2.0 * f.im) : mk(-2.0 * f.re, -2.0 * f.im);
        };
        sfor<0, R1>([&](auto Rr) QT_INL {
            const cx<double> ka = kfac(ln.ja + Rr * T), kb = kfac(ln.jb + Rr * T);
            a[Rr] = narrow(A[Rr] * ka);
            b[Rr] = narrow(B[Rr] * kb);
        });
        return;
    } else {
        constexpr int M = N / 2;
        using PH = Plan<M, W>;
        constexpr int H = PH::R1;           // = R1 / 2; the same T
        static_assert(PH::T == T && 2 * H == R1, "half-length plan");
        const Lanes<M, W> ln(opaque_lane(ln_in.t));
        const bool lane0 = ln.t == 0;
        // pairs (m, N - m) -> a+ (FP32) and a- (FP64) in the mirror layout of
        // length M.  Lanes t > 0: m = t + rT pairs with b[R1-1-r], m = T - t
        // + rT with a[R1-1-r].  Lane 0: m = rT pairs with (R1 - r) T
        // (itself at 0, where x = 0), m = W + rT with W + (R1-1-r) T.
        cx<float> ap[H], bp[H];
        cx<double> am[H], bm[H];
        sfor<0, H>([&](auto Rr) QT_INL {
            constexpr int r = Rr;
            ap[r] = a[r] + b[R1 - 1 - r];
            am[r] = widen(a[r]) - widen(b[R1 - 1 - r]);
            bp[r] = b[r] + a[R1 - 1 - r];
            bm[r] = widen(b[r]) - widen(a[R1 - 1 - r]);
        });
        // a+_M = x_{N/2} (lane 0, slot a[H] since N/2 = H T)
        const cx<float> apM = a[H];
        if (lane0) {
            sfor<0, H>([&](auto Rr) QT_INL {
                constexpr int r = Rr;
                constexpr int rm = (R1 - r) % R1;
                ap[r] = a[r] + a[rm];
                am[r] = widen(a[r]) - widen(a[rm]);
                bp[r] = b[r] + b[R1 - 1 - r];
                bm[r] = widen(b[r]) - widen(b[R1 - 1 - r]);
            });
        }
        // odd outputs: FFT input conj(V_j) = e^{-i pi j/N} (conj(a+_{M-j})
        // + i conj(a+_j)), in the mirror layout of length M (v[r] at
        // j = ja + rT, v[H + r] at j = jb + rT).  Lanes t > 0: the mirror
        // M - j of ja + rT is jb + (H-1-r) T and vice versa; lane 0: rT
        // pairs with (H - r) T, and V_0 = 2 a+_M.
        cx<float> v[PH::P];
        {
            const cx<float>* wd = opaque(tb.wd);
            sfor<0, H>([&](auto Rr) QT_INL {
                constexpr int r = Rr;
                v[r] = ldg(wd, ln.ja + r * T) * conj_plus_iconj(bp[H - 1 - r], ap[r]);
                v[H + r] = ldg(wd, ln.jb + r * T) * conj_plus_iconj(ap[H - 1 - r], bp[r]);
            });
            if (lane0) {
                sfor<0, H>([&](auto Rr) QT_INL {
                    constexpr int r = Rr;
                    if constexpr (r == 0) {
                        v[0] = mk(2.0f * apM.re, -2.0f * apM.im);
                    } else {
                        v[r] = ldg(wd, r * T) * conj_plus_iconj(ap[H - r], ap[r]);
                    }
                    v[H + r] = ldg(wd, W + r * T) * conj_plus_iconj(bp[H - 1 - r], bp[r]);
                });
            }
        }
        {
            PassTwiddles<float, M, W, 0> none;
            fft_passes<float, M, W, 0>(v, ln, static_cast<cx<float>*>(buf), opaque(tb.tw32), none);
        }
        // even outputs: dst1 of length M in FP64 (kinetic factors of F_{2q}
        // at M + q)
        {
            cx<double> pw[H];
            load_prew<double, M, W>(pw, tb.pre64h, ln);
            dst1<double, M, W, KIN>(am, bm, pw, tb.pre64h, ln, static_cast<cx<double>*>(buf), wsum,
                                    opaque(tb.tw64h),
                                    KIN ? reinterpret_cast<const Kin<double>*>(kin + M) : nullptr);
        }
        // every output to its place k in LDS, then back in the mirror layout
        // of length N.  Slot n = ja + rT of the cosine transform lies below
        // M/2 exactly when r < H/2 (ja, jb < T and (H/2) T = M/2).
        cx<float>* xb = static_cast<cx<float>*>(buf);
        sfor<0, H>([&](auto Rr) QT_INL {
            constexpr int r = Rr;
            constexpr bool low = r < H / 2;
            const int na = ln.ja + r * T, nb = ln.jb + r * T;
            const int ka = low ? 4 * na + 1 : 2 * N - 4 * na - 1;
            const int kb = low ? 4 * nb + 1 : 2 * N - 4 * nb - 1;
            const cx<float> fa = conjf(v[r]), fb = conjf(v[H + r]);
            if constexpr (KIN) {
                xb[pad(ka)] = mulk(fa, ldg(kin, (uint32_t)na));
                xb[pad(kb)] = mulk(fb, ldg(kin, (uint32_t)nb));
            } else {
                xb[pad(ka)] = low ? scale(fa, 0.5f) : scale(fa, -0.5f);
                xb[pad(kb)] = low ? scale(fb, 0.5f) : scale(fb, -0.5f);
            }
            xb[pad(2 * na)] = narrow(am[r]);
            xb[pad(2 * nb)] = narrow(bm[r]);
        });
        __syncthreads();
        const cx<float>* sa = xb + pad(ln_in.ja);
        const cx<float>* sb = xb + pad(ln_in.jb);
        sfor<0, R1>([&](auto Rr) QT_INL {
            a[Rr] = sa[padc<Rr * T>()];
            b[Rr] = sb[padc<Rr * T>()];
        });
        __syncthreads();
    }
}

}  // namespace qt
