// qt_eigen.cpp -- vacuum eigenstates of the discrete Hamiltonian (Sec.
// "Using the built-in eigensolvers"): 1S, 2S, 1P, 3S, 2P, 1D.
//
// H = T_kin + V on the grid r_m = m dr, m = 1..N-1, with T_kin diagonal in
// the sine modes (T_kin x = (2/N) S diag(E_k) S x, E_k of the derivative
// type) and V the vacuum singlet potential (Munich: -C_F alpha_s / r; KSU:
// the Cornell potential with string breaking) plus l(l+1)/(M r^2): the
// Hamiltonian the evolution integrates, at T = 0.  For each l the lowest
// states come from a locally optimal block preconditioned conjugate
// gradient iteration (LOBPCG, Knyazev 2001): the blocks live on the host
// (a few vectors of length N), H and the preconditioner (T_kin + sigma)^{-1}
// are applied on the GPU (eig_apply, two FP64 sine transforms per vector),
// and the Rayleigh-Ritz steps solve small dense symmetric eigenproblems
// with the cyclic Jacobi method.  Each state is normalised to
// dr sum u_m^2 = 1 with u_1 > 0.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "qt_host.hpp"

namespace qt {
namespace {

constexpr double kPiE = 3.14159265358979323846;

// Cyclic Jacobi eigen-decomposition of the symmetric n x n matrix a
// (row-major, destroyed): eigenvalues ascending in w, eigenvectors as the
// columns of v (row-major).
void jacobi_eig(int n, std::vector<double>& a, std::vector<double>& w, std::vector<double>& v)
{
    v.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double x = a[(size_t)i * n + j] * a[(size_t)i * n + j];
                tot += x;
                if (i != j) off += x;
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = a[(size_t)p * n + q];
                if (apq == 0.0) continue;
                const double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q];
                const double th = (aqq - app) / (2.0 * apq);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {          // columns p, q
                    const double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
                    a[(size_t)k * n + p] = c * akp - s * akq;
                    a[(size_t)k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {          // rows p, q
                    const double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
                    a[(size_t)p * n + k] = c * apk - s * aqk;
                    a[(size_t)q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = v[(size_t)k * n + p], vkq = v[(size_t)k * n + q];
                    v[(size_t)k * n + p] = c * vkp - s * vkq;
                    v[(size_t)k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    std::vector<int> ord(n);
    for (int i = 0; i < n; ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(),
              [&](int x, int y) { return a[(size_t)x * n + x] < a[(size_t)y * n + y]; });
    std::vector<double> v2((size_t)n * n);
    w.assign(n, 0.0);
    for (int j = 0; j < n; ++j) {
        w[j] = a[(size_t)ord[j] * n + ord[j]];
        for (int i = 0; i < n; ++i) v2[(size_t)i * n + j] = v[(size_t)i * n + ord[j]];
    }
    v.swap(v2);
}

double dot(const double* x, const double* y, int n)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += x[i] * y[i];
    return s;
}

// Rows of s (count x N) made orthonormal by two Cholesky-QR passes; false
// when the rows are (numerically) dependent.
bool orthonormalize(std::vector<double>& s, int count, int N)
{
    for (int pass = 0; pass < 2; ++pass) {
        std::vector<double> g((size_t)count * count);
        for (int i = 0; i < count; ++i)
            for (int j = 0; j <= i; ++j)
                g[(size_t)i * count + j] = g[(size_t)j * count + i] =
                    dot(&s[(size_t)i * N], &s[(size_t)j * N], N);
        double gmax = 0.0;
        for (int i = 0; i < count; ++i) gmax = std::max(gmax, g[(size_t)i * count + i]);
        // Cholesky g = L L^T, then rows <- L^{-1} rows
        std::vector<double> L((size_t)count * count, 0.0);
        for (int i = 0; i < count; ++i)
            for (int j = 0; j <= i; ++j) {
                double x = g[(size_t)i * count + j];
                for (int k = 0; k < j; ++k) x -= L[(size_t)i * count + k] * L[(size_t)j * count + k];
                if (i == j) {
                    if (!(x > 1e-13 * gmax)) return false;
                    L[(size_t)i * count + i] = std::sqrt(x);
                } else {
                    L[(size_t)i * count + j] = x / L[(size_t)j * count + j];
                }
            }
        for (int i = 0; i < count; ++i) {
            double* ri = &s[(size_t)i * N];
            for (int k = 0; k < i; ++k) {
                const double lik = L[(size_t)i * count + k];
                const double* rk = &s[(size_t)k * N];
                for (int m = 0; m < N; ++m) ri[m] -= lik * rk[m];
            }
            const double inv = 1.0 / L[(size_t)i * count + i];
            for (int m = 0; m < N; ++m) ri[m] *= inv;
        }
    }
    return true;
}

// y = sum_j c[j * ccols + col] x_j over the rows j < rows of x
void combine(const std::vector<double>& x, int rows, int N, const std::vector<double>& c, int ccols,
             int col, int row0, double* y)
{
    std::fill(y, y + N, 0.0);
    for (int j = row0; j < rows; ++j) {
        const double cj = c[(size_t)j * ccols + col];
        const double* xj = &x[(size_t)j * N];
        for (int m = 0; m < N; ++m) y[m] += cj * xj[m];
    }
}

// H and the preconditioner on the GPU for blocks of host vectors.
struct Operator {
    int N = 0;
    hipStream_t s = nullptr;
    double* dx = nullptr;
    double* dy = nullptr;
    double* dfh = nullptr;     // (2/N) E_k
    double* dfp = nullptr;     // (2/N) / (E_k + sigma)
    double* dv = nullptr;      // V_m (this l)
    void* tw = nullptr;        // FFT twiddles and DST-I weights of length N
    void* prew = nullptr;      // (its own: the context's caches are not locked here)
    int cap = 0;
    ~Operator()
    {
        hipFree(dx);
        hipFree(dy);
        hipFree(dfh);
        hipFree(dfp);
        hipFree(dv);
        hipFree(tw);
        hipFree(prew);
    }
    qt_status apply(const std::vector<double>& x, int count, bool precond, std::vector<double>& y)
    {
        y.assign((size_t)count * N, 0.0);
        if (count > cap) return fail(QT_EINVAL, "eigensolver block too large");
        QT_HIP(hipMemcpyAsync(dx, x.data(), (size_t)count * N * 8, hipMemcpyHostToDevice, s));
        QT_HIP(eig_apply(N, dx, dy, count, precond ? dfp : dfh, precond ? nullptr : dv, tw, prew, s));
        QT_HIP(hipMemcpyAsync(y.data(), dy, (size_t)count * N * 8, hipMemcpyDeviceToHost, s));
        QT_HIP(hipStreamSynchronize(s));
        return QT_OK;
    }
};

// The vacuum singlet potential plus the centrifugal term at r.
double vacuum_potential(const qt_physics* p, double r, int l)
{
    const double cent = (double)l * (l + 1) / (p->mass * r * r);
    if (p->potential == QT_POTENTIAL_KSU) {
        const double a = 0.409, sigma = 0.21, rsb = 1.25 / 0.1973269804;
        const double vsb = -a / rsb + sigma * rsb;
        return std::min(-a / r + sigma * r, vsb) + cent;
    }
    return -(4.0 / 3.0) * p->alpha_s / r + cent;
}

// The k lowest states of angular momentum l by LOBPCG; rows of u (k x N).
qt_status lowest_states(Operator& op, const qt_physics* p, int l, int k, double* lam,
                        std::vector<double>& u)
{
    const int N = p->N;
    const double dr = p->L / N;
    std::vector<double> V(N, 0.0);
    for (int m = 1; m < N; ++m) V[m] = vacuum_potential(p, m * dr, l);
    QT_HIP(hipMemcpyAsync(op.dv, V.data(), (size_t)N * 8, hipMemcpyHostToDevice, op.s));
    const int b = k + 2;
    // start: r^{l+1} e^{-r/rho_i}, rho_i growing with i (independent, smooth)
    const double a0 = p->alpha_s > 0.0 && p->potential != QT_POTENTIAL_KSU
                          ? 2.0 / (p->mass * (4.0 / 3.0) * p->alpha_s)
                          : 1.0;
    std::vector<double> X((size_t)b * N, 0.0);
    for (int i = 0; i < b; ++i)
        for (int m = 1; m < N; ++m) {
            const double r = m * dr;
            X[(size_t)i * N + m] = std::pow(r, l + 1) * std::exp(-r / (a0 * (l + 1 + 1.5 * i)));
        }
    if (!orthonormalize(X, b, N)) return fail(QT_ENOCONV, "eigensolver: dependent start");
    std::vector<double> AX, R, Wd, P, S, AS;
    qt_status st;
    if ((st = op.apply(X, b, false, AX)) != QT_OK) return st;
    double emax = 0.0;
    {
        // scale of H (largest kinetic energy plus the largest |V|) for the
        // residual tolerance: the transforms' rounding is relative to it
        std::vector<double> f(N);
        QT_HIP(hipMemcpy(f.data(), op.dfh, (size_t)N * 8, hipMemcpyDeviceToHost));
        for (int m = 1; m < N; ++m) emax = std::max(emax, std::fabs(f[m]) * N / 2 + std::fabs(V[m]));
    }
    const double tol = 1e-13 * emax;
    bool haveP = false;
    std::vector<double> w, C, G;
    for (int it = 0; it < 1000; ++it) {
        // Rayleigh-Ritz on span X
        G.assign((size_t)b * b, 0.0);
        for (int i = 0; i < b; ++i)
            for (int j = 0; j <= i; ++j)
                G[(size_t)i * b + j] = G[(size_t)j * b + i] =
                    0.5 * (dot(&X[(size_t)i * N], &AX[(size_t)j * N], N) +
                           dot(&X[(size_t)j * N], &AX[(size_t)i * N], N));
        jacobi_eig(b, G, w, C);
        {
            std::vector<double> X2((size_t)b * N), AX2((size_t)b * N);
            for (int i = 0; i < b; ++i) {
                combine(X, b, N, C, b, i, 0, &X2[(size_t)i * N]);
                combine(AX, b, N, C, b, i, 0, &AX2[(size_t)i * N]);
            }
            X.swap(X2);
            AX.swap(AX2);
        }
        R.assign((size_t)b * N, 0.0);
        double worst = 0.0;
        for (int i = 0; i < b; ++i) {
            double rn = 0.0;
            for (int m = 0; m < N; ++m) {
                const double x = AX[(size_t)i * N + m] - w[i] * X[(size_t)i * N + m];
                R[(size_t)i * N + m] = x;
                rn += x * x;
            }
            if (i < k) worst = std::max(worst, std::sqrt(rn));
        }
        if (worst <= tol) {
            for (int i = 0; i < k; ++i) lam[i] = w[i];
            u.assign(X.begin(), X.begin() + (size_t)k * N);
            return QT_OK;
        }
        if ((st = op.apply(R, b, true, Wd)) != QT_OK) return st;
        // S = [X; W; P]: X (orthonormal), then each row of W and P made
        // orthogonal to the rows before it (Gram-Schmidt, twice) and kept
        // only if a relative 1e-10 of it remains (a converged direction
        // drops out)
        S.assign(X.begin(), X.end());
        int ns = b;
        auto append = [&](const double* v) {
            std::vector<double> r(v, v + N);
            const double n0 = std::sqrt(dot(r.data(), r.data(), N));
            if (!(n0 > 0.0)) return;
            for (int pass = 0; pass < 2; ++pass)
                for (int j = 0; j < ns; ++j) {
                    const double* sj = &S[(size_t)j * N];
                    const double c = dot(sj, r.data(), N);
                    for (int m = 0; m < N; ++m) r[m] -= c * sj[m];
                }
            const double n1 = std::sqrt(dot(r.data(), r.data(), N));
            if (!(n1 > 1e-10 * n0) || ns >= op.cap) return;
            for (int m = 0; m < N; ++m) r[m] /= n1;
            S.insert(S.end(), r.begin(), r.end());
            ++ns;
        };
        for (int i = 0; i < b; ++i) append(&Wd[(size_t)i * N]);
        if (haveP)
            for (int i = 0; i < b; ++i) append(&P[(size_t)i * N]);
        if ((st = op.apply(S, ns, false, AS)) != QT_OK) return st;
        G.assign((size_t)ns * ns, 0.0);
        for (int i = 0; i < ns; ++i)
            for (int j = 0; j <= i; ++j)
                G[(size_t)i * ns + j] = G[(size_t)j * ns + i] =
                    0.5 * (dot(&S[(size_t)i * N], &AS[(size_t)j * N], N) +
                           dot(&S[(size_t)j * N], &AS[(size_t)i * N], N));
        jacobi_eig(ns, G, w, C);
        P.assign((size_t)b * N, 0.0);
        for (int i = 0; i < b; ++i) {
            combine(S, ns, N, C, ns, i, 0, &X[(size_t)i * N]);
            combine(AS, ns, N, C, ns, i, 0, &AX[(size_t)i * N]);
            combine(S, ns, N, C, ns, i, b, &P[(size_t)i * N]);
        }
        haveP = true;
    }
    return fail(QT_ENOCONV, "eigensolver did not converge (l = %d)", l);
}

}  // namespace

static qt_status eigen_basis(const qt_physics* p, double* energies, double* basis)
{
    const int N = p->N;
    if (!plain_supported(N)) return fail(QT_EINVAL, "N=%d not supported by the eigensolver", N);
    if (!(p->L > 0.0) || !(p->mass > 0.0)) return fail(QT_EINVAL, "L and mass must be positive");
    if (p->deriv_type != 0 && p->deriv_type != 1) return fail(QT_EINVAL, "deriv_type must be 0 or 1");
    if (p->potential != QT_POTENTIAL_MUNICH && p->potential != QT_POTENTIAL_KSU)
        return fail(QT_EINVAL, "unknown potential %d", p->potential);
    qt_status st = QT_OK;
    Operator op;
    op.N = N;
    op.cap = 15;                 // [X; W; P] for l = 0: 3 x (3 + 2)
    {
        std::vector<double> tw(2 * (size_t)N), sn(2 * (size_t)N);
        for (int m = 0; m < N; ++m) {
            tw[2 * m] = std::cos(2.0 * kPiE * m / N);
            tw[2 * m + 1] = -std::sin(2.0 * kPiE * m / N);
            const double sm = std::sin(kPiE * m / N);
            sn[2 * m] = 0.5 * (sm + 0.5);
            sn[2 * m + 1] = 0.5 * (sm - 0.5);
        }
        QT_HIP(hipMalloc(&op.tw, tw.size() * 8));
        QT_HIP(hipMalloc(&op.prew, sn.size() * 8));
        QT_HIP(hipMemcpy(op.tw, tw.data(), tw.size() * 8, hipMemcpyHostToDevice));
        QT_HIP(hipMemcpy(op.prew, sn.data(), sn.size() * 8, hipMemcpyHostToDevice));
    }
    QT_HIP(hipStreamCreateWithFlags(&op.s, hipStreamNonBlocking));
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() { hipStreamDestroy(s); }
    } guard{op.s};
    QT_HIP(hipMalloc(&op.dx, (size_t)op.cap * N * 8));
    QT_HIP(hipMalloc(&op.dy, (size_t)op.cap * N * 8));
    QT_HIP(hipMalloc(&op.dfh, (size_t)N * 8));
    QT_HIP(hipMalloc(&op.dfp, (size_t)N * 8));
    QT_HIP(hipMalloc(&op.dv, (size_t)N * 8));
    // kinetic factors; sigma = 1 GeV keeps the preconditioner positive
    // definite and leaves the low modes (the states sought) undamped
    std::vector<double> fh(N, 0.0), fp(N, 0.0);
    for (int k = 1; k < N; ++k) {
        const double e = kinetic_energy(p, k);
        fh[k] = (2.0 / N) * e;
        fp[k] = (2.0 / N) / (e + 1.0);
    }
    QT_HIP(hipMemcpy(op.dfh, fh.data(), (size_t)N * 8, hipMemcpyHostToDevice));
    QT_HIP(hipMemcpy(op.dfp, fp.data(), (size_t)N * 8, hipMemcpyHostToDevice));
    const double dr = p->L / N;
    static const int kSlots[3][3] = {{0, 1, 3}, {2, 4, -1}, {5, -1, -1}};
    static const int kCount[3] = {3, 2, 1};
    for (int l = 0; l < 3; ++l) {
        double lam[3];
        std::vector<double> u;
        if ((st = lowest_states(op, p, l, kCount[l], lam, u)) != QT_OK) return st;
        for (int i = 0; i < kCount[l]; ++i) {
            const int slot = kSlots[l][i];
            double* dst = basis + (size_t)slot * N;
            const double* src = &u[(size_t)i * N];
            double s2 = 0.0;
            for (int m = 1; m < N; ++m) s2 += src[m] * src[m];
            double f = 1.0 / std::sqrt(dr * s2);
            if (src[1] < 0.0) f = -f;
            dst[0] = 0.0;
            for (int m = 1; m < N; ++m) dst[m] = f * src[m];
            energies[slot] = lam[i];
        }
    }
    return QT_OK;
}

qt_status eigen_states(qt_context* ctx, const qt_physics* p, qt_context::Eigen* out)
{
    const std::vector<double> key{(double)p->N, p->L, p->mass, p->alpha_s, (double)p->deriv_type,
                                  (double)p->potential};
    std::lock_guard<std::mutex> lk(ctx->eig_mu);
    auto it = ctx->eigen.find(key);
    if (it != ctx->eigen.end()) {
        *out = it->second;
        return QT_OK;
    }
    if (g_no_alloc)
        return fail(QT_EINVAL, "vacuum eigenstates for this grid not computed on this context "
                    "yet: call qt_eigen_basis or qt_run with them first");
    QT_HIP(hipSetDevice(ctx->device));
    qt_context::Eigen e;
    auto b = std::make_shared<std::vector<double>>(6 * (size_t)p->N, 0.0);
    qt_status st = eigen_basis(p, e.energies, b->data());
    if (st != QT_OK) return st;
    e.basis = b;
    ctx->eigen[key] = e;
    *out = e;
    return QT_OK;
}

}  // namespace qt

extern "C" qt_status qt_eigen_basis(qt_context* ctx, const qt_physics* phys, double* energies,
                                    double* basis)
{
    if (!ctx || !phys || !energies || !basis) return qt::fail(QT_EINVAL, "null argument");
    qt_context::Eigen e;
    qt_status st = qt::eigen_states(ctx, phys, &e);
    if (st != QT_OK) return st;
    std::copy(e.energies, e.energies + 6, energies);
    std::copy(e.basis->begin(), e.basis->end(), basis);
    return QT_OK;
}
