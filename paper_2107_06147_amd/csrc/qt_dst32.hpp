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
// A step's kinetic block applies S K S; the second transform runs as the
// transpose of the first (kin_block32), so neither leaves its slots.
//
// Tables (one block, see ensure_tables): FP32 [e^{-i pi j/N}, j < M | the
// same in a second rounding], then FP64 [FFT twiddles of length M | DST-I
// weights of length M | FFT twiddles of length N | DST-I weights of length
// N], then the FP32 FFT twiddles of length M as level tables
// (PassTwiddles::load_level) in the two roundings.  The two roundings of the
// FP32 factors alternate step by step: their error, otherwise the same
// every step, then largely cancels between consecutive steps.  The kinetic
// factors are in the slot order of kin_block32 (below).
#pragma once
#include "qt_device.hpp"

namespace qt {

template <int N>
struct Dst32Tables {
    static constexpr int M = N / 2;
    const cx<float>* wd;       // e^{-i pi j / N}, j < M (rounding a or b)
    const cx<double>* tw64h;   // FFT twiddles, length M
    const cx<double>* pre64h;  // DST-I weights, length M
    const cx<double>* tw64;    // FFT twiddles, length N
    const cx<double>* pre64;   // DST-I weights, length N
    const cx<float>* lev32;    // FFT twiddles of length M, level table
    // the FP32 factors in rounding b when `second` (see ensure_tables)
    __device__ __forceinline__ Dst32Tables(const void* base, bool second)
    {
        const char* p = static_cast<const char*>(base);
        wd = reinterpret_cast<const cx<float>*>(p) + (second ? M : 0);
        tw64h = reinterpret_cast<const cx<double>*>(p + 2 * (size_t)M * sizeof(cx<float>));
        pre64h = tw64h + M;
        tw64 = pre64h + M;
        pre64 = tw64 + N;
        lev32 = reinterpret_cast<const cx<float>*>(pre64 + N) + (second ? level_table_len(M) : 0);
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

// LDS bytes of the exchange buffer that the FP32 kinetic block of length N
// on W lanes needs.
// (With eight or more values per lane: the FP64 buffer of length N/2, which
// also holds the two FP32 buffers of the cosine transform's FFTs.)
template <int N, int W>
constexpr size_t dst32_buf_bytes()
{
    return Plan<N, W>::P >= 8 ? sizeof(cx<double>) * (size_t)padded_len<N / 2>()
                              : sizeof(cx<double>) * (size_t)padded_len<N>();
}

// The kinetic block of a step, S diag(K) S x with S the DST-I of length N
// (S S = (N/2) I; K carries 2/N).  S = P diag(C, D) B: B the pair
// butterflies, C the cosine transform (odd outputs), D the half-length
// DST-I (even outputs), P the placement of the outputs by k.  S is
// symmetric, so the second transform is the transpose of the first, B^T
// diag(C^T, D^T) P^T, and P^T P = I: the outputs never leave the slots in
// which the first transform leaves them.  C^T: the same FFT (the DFT matrix
// is symmetric) and the transposed mixing, a+'_M = 2 U_0,
//   a+'_i = i conj(w_i) U_{M-i} - i w_i U_i   (w_i = e^{i pi i/N}),
// with U the inverse DFT of the slots; D^T = D; B^T = B.  With o = FFT(conj
// V) = conj(v) after the first FFT, the slot factor (1/2)^2 K_k of the
// odd outputs and U = conj(FFT(conj(u))) fold into one multiply of o by
// conj(K_k)/4 before the second FFT.  The kinetic table is in slot order:
// entry n < M is conj(K_k)/4 for the odd output k of slot n, entry M + q
// is K_{2q}.
// On entry a/b hold x in the mirror layout of length N, on exit the result
// in the same layout.  buf: LDS of dst32_buf_bytes<N, W>(); wsum: W/64
// cx<double> of LDS; odd_step selects the FP32 twiddles' second rounding.
// LEAN holds fewer values in registers across the block: each FFT pass's
// twiddles are loaded before its exchange (not all of them once for both
// FFTs), the mixing phases again for C^T, the kinetic factors of the even
// outputs where they are used.
template <int N, int W, bool LEAN = false>
__device__ __forceinline__ void kin_block32(cx<float>* a, cx<float>* b, const Lanes<N, W>& ln_in,
                                            void* buf, cx<double>* wsum, const void* tables,
                                            const cx<double>* __restrict__ kin, bool odd_step)
{
    using PL = Plan<N, W>;
    constexpr int R1 = PL::R1, T = PL::T;
    constexpr int M = N / 2;
    const Dst32Tables<N> tb(opaque(static_cast<const char*>(tables)), odd_step);
    if constexpr (PL::P < 8) {
        // widened: dst1 of length N in FP64, the kinetic factors in between
        // (natural order from the slot-ordered table)
        const Lanes<N, W> ln(opaque_lane(ln_in.t));
        cx<double> A[R1], B[R1], pw[R1];
        sfor<0, R1>([&](auto Rr) QT_INL {
            A[Rr] = widen(a[Rr]);
            B[Rr] = widen(b[Rr]);
        });
        load_prew<double, N, W>(pw, tb.pre64, ln);
        cx<double>* bd = static_cast<cx<double>*>(buf);
        dst1<double, N, W, false>(A, B, pw, tb.pre64, ln, bd, wsum, tb.tw64, nullptr);
        auto kfac = [&](int k) QT_INL {
            if ((k & 1) == 0) return ldg(kin, (uint32_t)(M + k / 2));
            const int n = ((k - 1) & 3) == 0 ? (k - 1) / 4 : (2 * N - 1 - k) / 4;
            const cx<double> f = ldg(kin, (uint32_t)n);
            return mk(4.0 * f.re, -4.0 * f.im);
        };
        sfor<0, R1>([&](auto Rr) QT_INL {
            A[Rr] = A[Rr] * kfac(ln.ja + Rr * T);
            B[Rr] = B[Rr] * kfac(ln.jb + Rr * T);
        });
        dst1<double, N, W, false>(A, B, pw, tb.pre64, ln, bd, wsum, opaque(tb.tw64), nullptr);
        sfor<0, R1>([&](auto Rr) QT_INL {
            a[Rr] = narrow(A[Rr]);
            b[Rr] = narrow(B[Rr]);
        });
    } else {
        using PH = Plan<M, W>;
        constexpr int H = PH::R1;           // = R1 / 2; the same T
        static_assert(PH::T == T && 2 * H == R1, "half-length plan");
        const Lanes<M, W> ln(opaque_lane(ln_in.t));
        const bool lane0 = ln.t == 0;
        // B: pairs (m, N - m) -> a+ (FP32) and a- (FP64) in the mirror layout
        // of length M.  Lanes t > 0: m = t + rT pairs with b[R1-1-r], m = T - t
        // + rT with a[R1-1-r].  Lane 0: m = rT pairs with (R1 - r) T (itself
        // at 0, where x = 0), m = W + rT with W + (R1-1-r) T.
        // (lane 0's partners are selected per lane, not taken in a branch:
        // the other waves of the workgroup would wait for it at the next
        // barrier)
        auto sel = [lane0](cx<float> p0, cx<float> p) QT_INL { return lane0 ? p0 : p; };
        cx<float> ap[H], bp[H];
        cx<double> am[H], bm[H];
        sfor<0, H>([&](auto Rr) QT_INL {
            constexpr int r = Rr;
            const cx<float> pa = sel(a[(R1 - r) % R1], b[R1 - 1 - r]);
            const cx<float> pb = sel(b[R1 - 1 - r], a[R1 - 1 - r]);
            ap[r] = a[r] + pa;
            am[r] = widen(a[r]) - widen(pa);
            bp[r] = b[r] + pb;
            bm[r] = widen(b[r]) - widen(pb);
        });
        // a+_M = x_{N/2} (lane 0, slot a[H] since N/2 = H T)
        const cx<float> apM = a[H];
        // C: FFT input conj(V_j) = e^{-i pi j/N} (conj(a+_{M-j}) + i
        // conj(a+_j)) in the mirror layout of length M (v[r] at j = ja + rT,
        // v[H + r] at j = jb + rT).  Lanes t > 0: the mirror M - j of ja + rT
        // is jb + (H-1-r) T and vice versa; lane 0: rT pairs with (H - r) T,
        // and V_0 = 2 a+_M.
        // e_j at this lane's slots (lane 0: ja = 0, jb = W), for C and C^T
        cx<float> ea[H], eb[H];
        {
            const cx<float>* wd = opaque(tb.wd);
            sfor<0, H>([&](auto Rr) QT_INL {
                ea[Rr] = ldg(wd, ln.ja + Rr * T);
                eb[Rr] = ldg(wd, ln.jb + Rr * T);
            });
        }
        cx<float> v[PH::P];
        sfor<0, H>([&](auto Rr) QT_INL {
            constexpr int r = Rr;
            v[r] = ea[r] * conj_plus_iconj(sel(ap[(H - r) % H], bp[H - 1 - r]), ap[r]);
            v[H + r] = eb[r] * conj_plus_iconj(sel(bp[H - 1 - r], ap[H - 1 - r]), bp[r]);
        });
        v[0] = sel(mk(2.0f * apM.re, -2.0f * apM.im), v[0]);
        // two exchange buffers (together the size of the FP64 one): the
        // first FFT exchanges through X, Y, X, ..., the second starts with
        // the other of the two that the first one ended on
        cx<float>* const bx = static_cast<cx<float>*>(buf);
        cx<float>* const by = bx + padded_len<M>();
        constexpr int NX = PH::NPASS - 1;   // exchanges per FFT
        // both FFTs take the same twiddles: loaded once (LEAN: per pass)
        AllTwiddles<float, M, W, LEAN ? Plan<M, W>::NPASS : 0> tws;
        const PassTwiddles<float, M, W, 0> none{};
        auto fft = [&](cx<float>* x, cx<float>* y) QT_INL {
            if constexpr (LEAN) fft_passes_db<float, M, W, 0>(v, ln, x, y, tb.lev32, none);
            else fft_passes_held<float, M, W, 0>(v, ln, x, y, tws);
        };
        if constexpr (!LEAN) tws.load_level(ln, opaque(tb.lev32));
        fft(bx, by);
        // slots n (v[r] at n = ja + rT, v[H + r] at jb + rT) times conj(K)/4
        {
            const cx<double>* kn = opaque(kin);
            sfor<0, H>([&](auto Rr) QT_INL {
                constexpr int r = Rr;
                v[r] = mulk(v[r], ldg(kn, (uint32_t)(ln.ja + r * T)));
                v[H + r] = mulk(v[H + r], ldg(kn, (uint32_t)(ln.jb + r * T)));
            });
        }
        if constexpr (NX % 2 == 1)
            fft(by, bx);
        else
            fft(bx, by);
        // the FP64 transforms below write the whole buffer
        __syncthreads();
        // C^T: U = conj(v); a+'_j = i (e_j U_{M-j} - conj(e_j) U_j), e_j =
        // e^{-i pi j/N}; a+'_M = 2 U_0 (lane 0)
        {
            auto tmix = [](cx<float> e, cx<float> um, cx<float> u) QT_INL {
                // i (e conj(um') - conj(e) conj(u')) with um', u' the FFT outputs
                const cx<float> p = e * conjf(um), q = conjf(e) * conjf(u);
                const cx<float> d = p - q;
                return mk(-d.im, d.re);
            };
            if constexpr (LEAN) {
                const cx<float>* wd = opaque(tb.wd);
                sfor<0, H>([&](auto Rr) QT_INL {
                    ea[Rr] = ldg(wd, ln.ja + Rr * T);
                    eb[Rr] = ldg(wd, ln.jb + Rr * T);
                });
            }
            sfor<0, H>([&](auto Rr) QT_INL {
                constexpr int r = Rr;
                ap[r] = tmix(ea[r], sel(v[(H - r) % H], v[H + H - 1 - r]), v[r]);
                bp[r] = tmix(eb[r], sel(v[H + H - 1 - r], v[H - 1 - r]), v[H + r]);
            });
            ap[0] = sel(mk(0.0f, 0.0f), ap[0]);
        }
        const cx<float> pM = mk(2.0f * v[0].re, -2.0f * v[0].im);
        // D, the kinetic factors of the even outputs, D^T = D, in FP64
        {
            cx<double> pw[H];
            load_prew<double, M, W>(pw, tb.pre64h, ln);
            cx<double>* b64 = static_cast<cx<double>*>(buf);
            dst1<double, M, W, true, LEAN>(am, bm, pw, tb.pre64h, ln, b64, wsum, opaque(tb.tw64h),
                                           reinterpret_cast<const Kin<double>*>(kin + M));
            dst1<double, M, W, false>(am, bm, pw, tb.pre64h, ln, b64, wsum, opaque(tb.tw64h),
                                      nullptr);
        }
        // B^T: x_m = a+'_m + a-'_m, x_{N-m} = a+'_m - a-'_m, x_{N/2} = a+'_M
        auto plus = [](cx<float> p, cx<double> q) QT_INL { return narrow(widen(p) + q); };
        auto minus = [](cx<float> p, cx<double> q) QT_INL { return narrow(widen(p) - q); };
        // every lane: x_m = a+'_m + a-'_m at its slots r < H of a and b; the
        // mirrors x_{N-m} = a+'_m - a-'_m go to b[R1-1-r] and a[R1-1-r], on
        // lane 0 to a[R1-r] and b[R1-1-r] (a[H] = x_{N/2}, a[0] = x_0 = 0)
        cx<float> ma[H], mb[H];
        sfor<0, H>([&](auto Rr) QT_INL {
            constexpr int r = Rr;
            a[r] = plus(ap[r], am[r]);
            b[r] = plus(bp[r], bm[r]);
            ma[r] = minus(ap[r], am[r]);
            mb[r] = minus(bp[r], bm[r]);
        });
        a[0] = sel(mk(0.0f, 0.0f), a[0]);
        sfor<H, R1>([&](auto Ii) QT_INL {
            constexpr int i = Ii;
            if constexpr (i == H) a[i] = sel(pM, mb[R1 - 1 - i]);
            else a[i] = sel(ma[R1 - i], mb[R1 - 1 - i]);
            b[i] = sel(mb[R1 - 1 - i], ma[R1 - 1 - i]);
        });
    }
}

}  // namespace qt
