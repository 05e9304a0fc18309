// qt_eigen.hip -- the operator kernel of the vacuum eigensolver.
//
// y = S (f .* (S x)) + d .* x for real vectors x of length N (index 0, the
// boundary, is 0), with S the DST-I (dst1, FP64) and f, d per-mode and
// per-point factors: f = (2/N) E_k and d = V gives H x, the discrete
// Hamiltonian of the evolution at T = 0 (Sec. "Using the built-in
// eigensolvers"); f = (2/N)/(E_k + sigma) and no d gives the
// preconditioner (T + sigma)^{-1}.  The sine transform is real, so one
// workgroup takes two real vectors as the real and imaginary parts of one
// complex vector.
#include "qt_device.hpp"
#include "qt_internal.h"

namespace qt {

template <int N, int W>
__global__ __launch_bounds__(W) void eig_apply_kernel(const double* __restrict__ x,
                                                      double* __restrict__ y, int n_vec,
                                                      const double* __restrict__ f,
                                                      const double* __restrict__ d,
                                                      const void* twv, const void* prewv)
{
    using PL = Plan<N, W>;
    constexpr int R1 = PL::R1, T = PL::T;
    __shared__ cx<double> buf[padded_len<N>()];
    __shared__ cx<double> wsum[W / 64];
    const int v0 = 2 * (int)blockIdx.x;
    const bool two = v0 + 1 < n_vec;
    const Lanes<N, W> ln(threadIdx.x);
    const double* xr = x + (size_t)v0 * N;
    const double* xi = xr + N;
    cx<double> a[R1], b[R1], a0[R1], b0[R1];
    sfor<0, R1>([&](auto Rr) QT_INL {
        const int ma = ln.ja + Rr * T, mb = ln.jb + Rr * T;
        a[Rr] = mk(xr[ma], two ? xi[ma] : 0.0);
        b[Rr] = mk(xr[mb], two ? xi[mb] : 0.0);
        a0[Rr] = a[Rr];
        b0[Rr] = b[Rr];
    });
    const cx<double>* prew = static_cast<const cx<double>*>(prewv);
    const cx<double>* tw = static_cast<const cx<double>*>(twv);
    cx<double> pw[R1];
    load_prew<double, N, W>(pw, prew, ln);
    dst1<double, N, W, false>(a, b, pw, prew, ln, buf, wsum, tw, nullptr);
    sfor<0, R1>([&](auto Rr) QT_INL {
        a[Rr] = scale(a[Rr], f[ln.ja + Rr * T]);
        b[Rr] = scale(b[Rr], f[ln.jb + Rr * T]);
    });
    dst1<double, N, W, false>(a, b, pw, prew, ln, buf, wsum, tw, nullptr);
    if (d != nullptr) {
        sfor<0, R1>([&](auto Rr) QT_INL {
            a[Rr] = a[Rr] + scale(a0[Rr], d[ln.ja + Rr * T]);
            b[Rr] = b[Rr] + scale(b0[Rr], d[ln.jb + Rr * T]);
        });
    }
    double* yr = y + (size_t)v0 * N;
    double* yi = yr + N;
    sfor<0, R1>([&](auto Rr) QT_INL {
        const int ma = ln.ja + Rr * T, mb = ln.jb + Rr * T;
        yr[ma] = a[Rr].re;
        yr[mb] = b[Rr].re;
        if (two) {
            yi[ma] = a[Rr].im;
            yi[mb] = b[Rr].im;
        }
    });
}

template <int N, int W>
static hipError_t eig_apply_n(const double* x, double* y, int n_vec, const double* f,
                              const double* d, const void* tw, const void* prew, hipStream_t s)
{
    hipLaunchKernelGGL((eig_apply_kernel<N, W>), dim3((unsigned)((n_vec + 1) / 2)), dim3(W), 0, s,
                       x, y, n_vec, f, d, tw, prew);
    return hipGetLastError();
}

hipError_t eig_apply(int N, const double* x, double* y, int n_vec, const double* f,
                     const double* d, const void* tw, const void* prew, hipStream_t s)
{
    if (n_vec <= 0) return hipSuccess;
    switch (N) {
    case 256: return eig_apply_n<256, 64>(x, y, n_vec, f, d, tw, prew, s);
    case 512: return eig_apply_n<512, 64>(x, y, n_vec, f, d, tw, prew, s);
    case 1024: return eig_apply_n<1024, 128>(x, y, n_vec, f, d, tw, prew, s);
    case 2048: return eig_apply_n<2048, 256>(x, y, n_vec, f, d, tw, prew, s);
    case 4096: return eig_apply_n<4096, 256>(x, y, n_vec, f, d, tw, prew, s);
    case 8192: return eig_apply_n<8192, 512>(x, y, n_vec, f, d, tw, prew, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace qt
