// qt_api.cpp -- C ABI entry points, validation and host-side setup.
//
// Host setup follows the paper's statement of the problem (table "Code
// parameters"; Secs. "Derivative types", "Algorithm for deterministic
// evolution between quantum jumps"; appendix "Munich potential"):
// the kinetic factors exp(-i T_kin dt) on the momentum grid p_k = pi k/L,
// the initial state normalised with eq. (normcond), the hydrogen-like
// Coulomb basis used for the overlaps, and the number of steps the
// temperature table allows.  Everything here is FP64; the FP32-bulk form
// rounds each table once when it is uploaded.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "qt_host.hpp"
#include "qt_philox.h"

namespace {
thread_local std::string g_last_error;
constexpr double kPi = 3.14159265358979323846;
}  // namespace

namespace qt {
thread_local bool g_no_alloc = false;

bool trace_on()
{
    const char* e = std::getenv("QTRAJ_TRACE");
    return e && *e;
}

void trace_line(const char* fmt, ...)
{
    static std::mutex mu;
    const char* e = std::getenv("QTRAJ_TRACE");
    if (!e || !*e) return;
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    std::lock_guard<std::mutex> lk(mu);
    const bool err = std::strcmp(e, "stderr") == 0 || std::strcmp(e, "-") == 0;
    FILE* f = err ? stderr : std::fopen(e, "a");
    if (!f) return;
    std::fprintf(f, "%s\n", buf);
    if (err) std::fflush(f);
    else std::fclose(f);
}
}  // namespace qt

namespace qt {

qt_status fail(qt_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

int elem_bytes(int prec) { return prec == QT_FP32_BULK ? 8 : 16; }

// ---------------------------------------------------------------- setup ---

double host_temperature(const double* tau, const double* T, int n, double t)
{
    if (t <= tau[0]) return T[0];
    if (t >= tau[n - 1]) return T[n - 1];
    int i = 0;
    while (!(tau[i + 1] > t)) ++i;
    const double w = (t - tau[i]) / (tau[i + 1] - tau[i]);
    return T[i] + (T[i + 1] - T[i]) * w;
}

int64_t count_steps(const qt_physics& p, const qt_ttable& tt)
{
    // The step count stops where the table ends or T(t_n) drops below
    // T_final, with t_n = tau_start + n dt and T linear between the table's
    // points (the interpolation the kernels use).  Steps are
    // taken one by one only where that decision can go either way: a run of
    // steps before the table or inside one of its intervals is passed at
    // once when T there cannot fall below T_final (both ends of the
    // interval above it by more than the interpolation's rounding).  t_n
    // grows with n, so the first step past a point is found by an estimate
    // and a correction.
    const double* tau = tt.tau;
    const double* Tt = tt.T;
    const int last = tt.n - 1;
    auto t_of = [&](int64_t n) { return tt.tau_start + (double)n * p.dt; };
    // first n' > n with t_{n'} >= x (ge) or t_{n'} > x (!ge)
    auto first_past = [&](int64_t n, double x, bool ge) {
        auto past = [&](int64_t k) { return ge ? t_of(k) >= x : t_of(k) > x; };
        const double est = std::ceil((x - tt.tau_start) / p.dt);
        // (the estimate is off by a step at most: beyond the cap is beyond it)
        if (est >= (double)tt.max_steps + 2.0) return tt.max_steps;
        int64_t k = est > (double)n + 1.0 ? (int64_t)est : n + 1;
        while (k > n + 1 && past(k - 1)) --k;
        while (!past(k)) ++k;
        return k;
    };
    const double eps = 4.0 * 2.220446049250313e-16;
    int64_t n = 0;
    int i = 0;
    while (n < tt.max_steps) {
        const double t = t_of(n);
        if (t > tau[last]) break;
        double T;
        if (t <= tau[0]) {
            if (Tt[0] >= tt.T_final) {
                n = std::min(first_past(n, tau[0], false), tt.max_steps);
                continue;
            }
            T = Tt[0];
        } else if (t >= tau[last]) {
            T = Tt[last];
        } else {
            while (!(tau[i + 1] > t)) ++i;
            const double lo = std::min(Tt[i], Tt[i + 1]);
            if (lo - eps * (std::fabs(Tt[i]) + std::fabs(Tt[i + 1])) >= tt.T_final) {
                n = std::min(first_past(n, tau[i + 1], true), tt.max_steps);
                continue;
            }
            const double w = (t - tau[i]) / (tau[i + 1] - tau[i]);
            T = Tt[i] + (Tt[i + 1] - Tt[i]) * w;
        }
        if (T < tt.T_final) break;
        ++n;
    }
    return n;
}

static bool coulomb_state_known(int n, int l)
{
    return (n == 1 && l == 0) || (n == 2 && (l == 0 || l == 1)) ||
           (n == 3 && (l >= 0 && l <= 2));
}

static qt_status validate_ttable(const qt_ttable* tt)
{
    if (!tt->tau || !tt->T || tt->n < 2) return fail(QT_EINVAL, "temperature table needs >= 2 points");
    for (int i = 0; i + 1 < tt->n; ++i)
        if (!(tt->tau[i + 1] > tt->tau[i])) return fail(QT_EINVAL, "tau must increase strictly");
    for (int i = 0; i < tt->n; ++i)
        if (!(tt->T[i] >= 0) || !std::isfinite(tt->T[i])) return fail(QT_EINVAL, "T must be finite and >= 0");
    if (tt->max_steps < 0) return fail(QT_EINVAL, "max_steps must be >= 0");
    if (!std::isfinite(tt->tau_start)) return fail(QT_EINVAL, "tau_start must be finite");
    return QT_OK;
}

qt_status validate(const qt_physics* p, const qt_ttable* tt, const qt_init* in, const qt_batch* b)
{
    if (!p || !tt || !in || !b) return fail(QT_EINVAL, "null argument");
    if (p->N < 256 || p->N > 8192 || (p->N & (p->N - 1)) != 0)
        return fail(QT_EINVAL, "N = %d: must be a power of two in [256, 8192]", p->N);
    if (!(p->L > 0) || !(p->dt > 0) || !(p->mass > 0))
        return fail(QT_EINVAL, "L, dt and mass must be > 0");
    if (!(p->alpha_s >= 0)) return fail(QT_EINVAL, "alpha_s must be >= 0");
    if (!(p->kappa_hat >= 0 || p->kappa_hat == -1.0 || p->kappa_hat == -2.0 || p->kappa_hat == -3.0))
        return fail(QT_EINVAL, "kappa_hat must be >= 0, or -1/-2/-3 for a fit");
    if (!(p->gamma_hat <= 0)) return fail(QT_EINVAL, "gamma_hat must be <= 0");
    if (p->deriv_type != 0 && p->deriv_type != 1) return fail(QT_EINVAL, "deriv_type must be 0 or 1");
    if (!(p->r_max > 0) || p->r_max > 1) return fail(QT_EINVAL, "r_max must be in (0, 1]");
    if (p->flags & ~QT_FLAG_KINETIC_OFF) return fail(QT_EINVAL, "unknown flags 0x%x", p->flags);
    if (qt_status st = validate_ttable(tt); st != QT_OK) return st;
    if (in->l < 0 || in->l > 1000) return fail(QT_EINVAL, "initial l out of range");
    if (in->color != QT_SINGLET && in->color != QT_OCTET) return fail(QT_EINVAL, "color must be 0 or 1");
    switch (in->kind) {
    case QT_INIT_COULOMB:
        if (!(p->alpha_s > 0)) return fail(QT_EINVAL, "Coulomb initial state needs alpha_s > 0");
        if (!coulomb_state_known(in->n, in->l))
            return fail(QT_EINVAL, "Coulomb state (n=%d, l=%d) not available (n <= 3)", in->n, in->l);
        break;
    case QT_INIT_GAUSSIAN:
        if (!(in->width > 0)) return fail(QT_EINVAL, "Gaussian width must be > 0");
        break;
    case QT_INIT_ARRAY:
        if (!in->u_re) return fail(QT_EINVAL, "array initial state needs u_re");
        break;
    case QT_INIT_EIGEN:
        if (in->color != QT_SINGLET) return fail(QT_EINVAL, "eigenstate initial states are singlets");
        if (!coulomb_state_known(in->n, in->l))
            return fail(QT_EINVAL, "eigenstate (n=%d, l=%d) not computed (1S..1D)", in->n, in->l);
        break;
    default: return fail(QT_EINVAL, "unknown initial state kind %d", in->kind);
    }
    if (b->n_traj < 0 || b->n_traj > 0x7fffffffLL) return fail(QT_EINVAL, "n_traj out of range");
    if (b->precision != QT_FP64 && b->precision != QT_FP32_BULK)
        return fail(QT_EINVAL, "unknown precision %d", b->precision);
    if (b->form != QT_FORM_FUSED && b->form != QT_FORM_PLAIN)
        return fail(QT_EINVAL, "unknown form %d", b->form);
    if (b->form == QT_FORM_PLAIN && b->precision != QT_FP64)
        return fail(QT_EINVAL, "the plain form is FP64 only");
    if (tt->vacuum_steps < 0) return fail(QT_EINVAL, "vacuum_steps must be >= 0");
    if (p->potential != QT_POTENTIAL_MUNICH && p->potential != QT_POTENTIAL_KSU)
        return fail(QT_EINVAL, "unknown potential %d", p->potential);
    if (p->basis != QT_BASIS_COULOMB && p->basis != QT_BASIS_EIGEN)
        return fail(QT_EINVAL, "unknown basis %d", p->basis);
    if (p->potential == QT_POTENTIAL_KSU) {
        if (p->do_jumps) return fail(QT_EINVAL, "the KSU potential runs without jumps");
        if (in->color != QT_SINGLET) return fail(QT_EINVAL, "the KSU potential is a singlet potential");
        if (!(p->md_factor > 0) || !std::isfinite(p->md_factor))
            return fail(QT_EINVAL, "md_factor must be > 0");
    }
    if (b->no_jump_shortcut != 0 && b->no_jump_shortcut != 1)
        return fail(QT_EINVAL, "no_jump_shortcut must be 0 or 1");
    if (b->no_jump_shortcut && b->form != QT_FORM_FUSED)
        return fail(QT_EINVAL, "the no-jump shortcut runs in the fused form");
    // the rMin test precedes the rMax test; rMin is known only once the
    // zeroth trajectory has run, so the shortcut needs rMax = 1
    if (b->no_jump_shortcut && p->r_max != 1.0)
        return fail(QT_EINVAL, "the no-jump shortcut needs r_max = 1");
    return QT_OK;
}

// u = r R_nl of the hydrogen-like problem with Bohr radius a0 (reduced mass
// M/2: a0 = 2/(M alpha)); normalisation is redone on the grid.
static double hydrogen(int n, int l, double a0, double r)
{
    const double x = r / a0;
    switch (n * 10 + l) {
    case 10: return r * std::exp(-x);
    case 20: return r * (1.0 - 0.5 * x) * std::exp(-0.5 * x);
    case 21: return r * r * std::exp(-0.5 * x);
    case 30: return r * (1.0 - 2.0 * x / 3.0 + 2.0 * x * x / 27.0) * std::exp(-x / 3.0);
    case 31: return r * r * (1.0 - x / 6.0) * std::exp(-x / 3.0);
    case 32: return r * r * r * std::exp(-x / 3.0);
    }
    return 0.0;
}

static void normalise(std::vector<double>& u, int N, double dr, bool complex_pairs)
{
    double s = 0.0;
    const int stride = complex_pairs ? 2 : 1;
    for (int j = 1; j < N; ++j)
        for (int c = 0; c < stride; ++c) s += u[stride * j + c] * u[stride * j + c];
    if (!(s > 0)) return;
    const double f = 1.0 / std::sqrt(dr * s);
    for (double& v : u) v *= f;
}

// Process-wide cache of host tables keyed by the parameters they depend on.
// Entries live as long as some batch holds them.
template <class T>
class TableCache {
public:
    template <class Make>
    std::shared_ptr<const T> get(const std::vector<double>& key, Make make)
    {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = m_.find(key);
        if (it != m_.end()) {
            if (auto sp = it->second.lock()) return sp;
        }
        if (m_.size() > 256) {
            for (auto i = m_.begin(); i != m_.end();) i = i->second.expired() ? m_.erase(i) : std::next(i);
        }
        std::shared_ptr<const T> sp = make();
        if (sp) m_[key] = sp;
        return sp;
    }

private:
    std::mutex mu_;
    std::map<std::vector<double>, std::weak_ptr<const T>> m_;
};

static const int kBasisN[6] = {1, 2, 2, 3, 3, 3}, kBasisL[6] = {0, 0, 1, 0, 1, 2};

// kinetic energy of sine mode k (Sec. "Derivative types"): p_k^2 / M, or
// 2 (1 - cos(p_k dr)) / (M dr^2) for derivType 1, p_k = pi k / L
double kinetic_energy(const qt_physics* p, int k)
{
    const double dr = p->L / p->N;
    const double pk = kPi * k / p->L;
    return p->deriv_type == 1 ? 2.0 * (1.0 - std::cos(pk * dr)) / (p->mass * dr * dr)
                              : pk * pk / p->mass;
}

// kinetic factors (2/N) exp(-i E_k dt); 2/N is the scale of two
// unnormalised sine transforms
static std::shared_ptr<const std::vector<double>> kinetic_table(const qt_physics* p)
{
    static TableCache<std::vector<double>> cache;
    const int N = p->N;
    const int off = (p->flags & QT_FLAG_KINETIC_OFF) ? 1 : 0;
    const std::vector<double> key{(double)N, p->L, p->dt, p->mass, (double)p->deriv_type, (double)off};
    return cache.get(key, [&] {
        const double dr = p->L / N;
        auto t = std::make_shared<std::vector<double>>(2 * (size_t)N, 0.0);
        for (int k = 1; k < N; ++k) {
            double re = 1.0, im = 0.0;
            if (!off) {
                const double E = kinetic_energy(p, k);
                re = std::cos(E * p->dt);
                im = -std::sin(E * p->dt);
            }
            (*t)[2 * k] = (2.0 / N) * re;
            (*t)[2 * k + 1] = (2.0 / N) * im;
        }
        return std::shared_ptr<const std::vector<double>>(t);
    });
}

// Coulomb basis 1S, 2S, 1P, 3S, 2P, 1D (zero when alpha_s = 0)
static std::shared_ptr<const std::vector<double>> basis_table(const qt_physics* p)
{
    static TableCache<std::vector<double>> cache;
    const int N = p->N;
    const std::vector<double> key{(double)N, p->L, p->mass, p->alpha_s};
    return cache.get(key, [&] {
        const double dr = p->L / N;
        auto t = std::make_shared<std::vector<double>>(6 * (size_t)N, 0.0);
        if (p->alpha_s > 0) {
            const double a0 = 2.0 / (p->mass * (4.0 / 3.0) * p->alpha_s);
            for (int q = 0; q < 6; ++q) {
                std::vector<double> u(N, 0.0);
                for (int j = 1; j < N; ++j) u[j] = hydrogen(kBasisN[q], kBasisL[q], a0, j * dr);
                normalise(u, N, dr, false);
                std::copy(u.begin(), u.end(), t->begin() + (size_t)q * N);
            }
        }
        return std::shared_ptr<const std::vector<double>>(t);
    });
}

// Initial state and its overlaps; null if its norm is zero or not finite.
static std::shared_ptr<const InitTable> make_init(const qt_physics* p, const qt_init* in,
                                                  const std::vector<double>& basis,
                                                  const std::vector<double>* eigen)
{
    const int N = p->N;
    const double dr = p->L / N;
    auto t = std::make_shared<InitTable>();
    std::vector<double>& psi = t->psi;
    psi.assign(2 * (size_t)N, 0.0);
    if (in->kind == QT_INIT_COULOMB) {
        const double a0 = 2.0 / (p->mass * (4.0 / 3.0) * p->alpha_s);
        for (int j = 1; j < N; ++j) psi[2 * j] = hydrogen(in->n, in->l, a0, j * dr);
    } else if (in->kind == QT_INIT_EIGEN) {
        int q = 0;
        while (kBasisN[q] != in->n || kBasisL[q] != in->l) ++q;
        for (int j = 1; j < N; ++j) psi[2 * j] = (*eigen)[(size_t)q * N + j];
    } else if (in->kind == QT_INIT_GAUSSIAN) {
        for (int j = 1; j < N; ++j) {
            const double r = j * dr;
            psi[2 * j] = std::pow(r, (double)(in->l + 1)) * std::exp(-r * r / (2.0 * in->width * in->width));
        }
    } else {
        for (int j = 1; j < N; ++j) {
            psi[2 * j] = in->u_re[j];
            psi[2 * j + 1] = in->u_im ? in->u_im[j] : 0.0;
        }
    }
    double s = 0.0;
    for (int j = 1; j < N; ++j) s += psi[2 * j] * psi[2 * j] + psi[2 * j + 1] * psi[2 * j + 1];
    if (!(s > 0) || !std::isfinite(s)) return nullptr;
    normalise(psi, N, dr, true);

    // initial overlaps |<b|u>|^2/<u|u> (singlet of matching l only)
    double nrm = 0.0;
    for (int j = 1; j < N; ++j) nrm += psi[2 * j] * psi[2 * j] + psi[2 * j + 1] * psi[2 * j + 1];
    for (int q = 0; q < 6; ++q) {
        t->overlap[q] = 0.0;
        if (in->color != QT_SINGLET || in->l != kBasisL[q]) continue;
        if (p->basis == QT_BASIS_COULOMB && !(p->alpha_s > 0)) continue;
        double ar = 0.0, ai = 0.0;
        for (int j = 1; j < N; ++j) {
            ar += basis[(size_t)q * N + j] * psi[2 * j];
            ai += basis[(size_t)q * N + j] * psi[2 * j + 1];
        }
        ar *= dr;
        ai *= dr;
        t->overlap[q] = (ar * ar + ai * ai) / (dr * nrm);
    }
    return t;
}

qt_status prepare(qt_context* ctx, const qt_physics* p, const qt_ttable* tt, const qt_init* in,
                  const qt_batch* b, HostBatch* hb)
{
    qt_status st = validate(p, tt, in, b);
    if (st != QT_OK) return st;
    // the vacuum eigenstates (ProjType 1, initType 100), computed on the
    // device once per context and parameters
    qt_context::Eigen eig;
    if (p->basis == QT_BASIS_EIGEN || in->kind == QT_INIT_EIGEN) {
        if (!ctx) return fail(QT_EINVAL, "eigenstates need a context");
        if ((st = eigen_states(ctx, p, &eig)) != QT_OK) return st;
    }
    hb->phys = *p;
    hb->batch = *b;
    hb->init_l = in->l;
    hb->init_color = in->color;
    hb->tau.assign(tt->tau, tt->tau + tt->n);
    hb->T.assign(tt->T, tt->T + tt->n);
    hb->tau_start = tt->tau_start;
    hb->T_final = tt->T_final;
    hb->n_steps = count_steps(*p, *tt);
    hb->vacuum_steps = tt->vacuum_steps;
    hb->kin = kinetic_table(p);
    hb->basis = p->basis == QT_BASIS_EIGEN ? eig.basis : basis_table(p);
    const std::vector<double>* ev = eig.basis ? eig.basis.get() : nullptr;
    if (in->kind == QT_INIT_ARRAY) {
        hb->init = make_init(p, in, *hb->basis, ev);
    } else {
        static TableCache<InitTable> cache;
        const std::vector<double> key{(double)p->N, p->L, p->mass, p->alpha_s, (double)in->kind,
                                      (double)in->n, (double)in->l, (double)in->color, in->width,
                                      (double)p->basis, (double)p->deriv_type,
                                      (double)p->potential};
        hb->init = cache.get(key, [&] { return make_init(p, in, *hb->basis, ev); });
    }
    if (!hb->init) return fail(QT_EINVAL, "initial state has zero or non-finite norm");
    return QT_OK;
}

// -------------------------------------------------- per-N device tables ---

qt_status ensure_tables(qt_context* ctx, int prec, int N, qt_context::Tables* out)
{
    auto key = std::make_pair(prec, N);
    auto it = ctx->tables.find(key);
    if (it != ctx->tables.end()) {
        *out = it->second;
        return QT_OK;
    }
    if (g_no_alloc)
        return fail(QT_EINVAL, "no transform tables for N=%d precision=%d on this context yet: "
                    "run qt_run with this grid first", N, prec);
    const bool f32 = prec == QT_FP32_BULK;
    // FFT twiddles exp(-2 pi i m/n) and DST-I pre-processing weights
    // ((s + 1/2)/2, (s - 1/2)/2), s = sin(pi m/n), of a transform of length n
    auto fill = [](int n, double* tw, double* sn) {
        for (int m = 0; m < n; ++m) {
            tw[2 * m] = std::cos(2.0 * kPi * m / n);
            tw[2 * m + 1] = -std::sin(2.0 * kPi * m / n);
            const double s = std::sin(kPi * m / n);
            sn[2 * m] = 0.5 * (s + 0.5);
            sn[2 * m + 1] = 0.5 * (s - 0.5);
        }
    };
    qt_context::Tables t;
    if (f32) {
        // the FP32 sine transform (split form, qt_dst32.hpp), one block:
        // FP32 [exp(-i pi j/N), j < M = N/2, rounding a | the same in
        // rounding b], FP64 [FFT twiddles, DST-I weights of length M | the
        // same of length N], then the FP32 FFT twiddles of length M as level
        // tables (rounding a | rounding b): level L = 4, 8, ..., M holds
        // exp(-2 pi i r k / L), r = 1..7, k < L/2, in pair rows
        // (level_index), so that the lanes of an FFT pass read consecutive
        // entries.
        // Rounding a is to nearest; b rounds 2w - a, so that (a + b)/2 lies
        // closer to w than either.  The kernel alternates the two step by
        // step: the rounding error of these factors, the same every step
        // with one table, then largely cancels between consecutive steps
        // instead of adding up.
        // (The neighbour of modulus closest to 1 would trade the modulus
        // error for a larger phase error, which adds up the same way.)
        const int M = N / 2;
        const size_t nl = (size_t)level_table_len(M);
        const size_t f0 = 4 * (size_t)M;        // floats of the mixing phases
        std::vector<float> f(f0 + 4 * nl);
        auto two = [&](size_t ia, size_t ib, double c, double s) {
            f[2 * ia] = (float)c;
            f[2 * ia + 1] = (float)s;
            f[2 * ib] = (float)(2.0 * c - (double)f[2 * ia]);
            f[2 * ib + 1] = (float)(2.0 * s - (double)f[2 * ia + 1]);
        };
        for (int m = 0; m < M; ++m)
            two(m, (size_t)M + m, std::cos(kPi * m / N), -std::sin(kPi * m / N));
        for (int L = 4; L <= M; L *= 2)
            for (int r = 1; r <= 7; ++r)
                for (int k = 0; k < L / 2; ++k) {
                    const int m = (int)(((int64_t)r * k) % L);
                    const size_t e = (size_t)level_index(L, r, k);
                    two(f0 / 2 + e, f0 / 2 + nl + e, std::cos(2.0 * kPi * m / L),
                        -std::sin(2.0 * kPi * m / L));
                }
        std::vector<double> d(4 * (size_t)M + 4 * (size_t)N);
        fill(M, &d[0], &d[2 * (size_t)M]);
        fill(N, &d[4 * (size_t)M], &d[4 * (size_t)M + 2 * (size_t)N]);
        QT_HIP(hipMalloc(&t.tw, f.size() * 4 + d.size() * 8));
        QT_HIP(hipMemcpy(t.tw, f.data(), f0 * 4, hipMemcpyHostToDevice));
        QT_HIP(hipMemcpy(static_cast<char*>(t.tw) + f0 * 4, d.data(), d.size() * 8,
                         hipMemcpyHostToDevice));
        QT_HIP(hipMemcpy(static_cast<char*>(t.tw) + f0 * 4 + d.size() * 8, f.data() + f0,
                         (f.size() - f0) * 4, hipMemcpyHostToDevice));
        t.prew = nullptr;
    } else {
        std::vector<double> tw(2 * (size_t)N), sn(2 * (size_t)N);
        fill(N, tw.data(), sn.data());
        QT_HIP(hipMalloc(&t.tw, 2 * N * 8));
        QT_HIP(hipMalloc(&t.prew, 2 * N * 8));
        QT_HIP(hipMemcpy(t.tw, tw.data(), tw.size() * 8, hipMemcpyHostToDevice));
        QT_HIP(hipMemcpy(t.prew, sn.data(), sn.size() * 8, hipMemcpyHostToDevice));
    }
    ctx->tables[key] = t;
    *out = t;
    return QT_OK;
}

// ------------------------------------------------ KSU phi(r-hat) table ---
//
// phi(a) = 2 int_0^inf dz z/(z^2+1)^2 [1 - sin(z a)/(z a)] of the KSU
// potential's imaginary part (appendix "Isotropic KSU potential").  With
// I(a) = int_0^inf sin(a z)/(1+z^2)^2 dz, phi = 1 - 2 I/a, and from the sine
// integral of 1/(z^2+b^2) in terms of the exponential integral,
// differentiated in b at b = 1:
//   I(a)  = [(a+1) e^{-a} Ei(a) + (a-1) e^{a} Ei(-a)] / 4,
//   I'(a) = [2 - a e^{-a} Ei(a) + a e^{a} Ei(-a)] / 4,
//   phi'(a) = 2 I/a^2 - 2 I'/a.
// Table: (phi, phi') at a = k/8192, k = 0..4096, then at a = 1/2 + k/256,
// k = 0..16256, for cubic Hermite interpolation on the device.

// e^{-a} Ei(a), a > 0 (power series of Ei, positive terms)
static double scaled_ei(double a)
{
    double t = 1.0, s = 0.0;
    for (int k = 1; k < 2000; ++k) {
        t *= a / k;
        const double d = t / k;
        s += d;
        if (d <= 1e-18 * s) break;
    }
    return std::exp(-a) * (0.5772156649015328606 + std::log(a) + s);
}

// e^{a} E1(a) = -e^{a} Ei(-a), a > 0: series below 1, continued fraction
// (modified Lentz) above
static double scaled_e1(double a)
{
    if (a < 1.0) {
        double t = 1.0, s = 0.0;        // sum_k (-a)^k / (k k!)
        for (int k = 1; k < 40; ++k) {
            t *= -a / k;
            s += t / k;
        }
        return std::exp(a) * (-0.5772156649015328606 - std::log(a) - s);
    }
    const double tiny = 1e-300;
    double b = a + 1.0, c = 1.0 / tiny, d = 1.0 / b, h = d;
    for (int i = 1; i < 10000; ++i) {
        const double an = -(double)i * i;
        b += 2.0;
        d = 1.0 / (an * d + b);
        c = b + an / c;
        const double del = c * d;
        h *= del;
        if (std::fabs(del - 1.0) < 1e-16) break;
    }
    return h;
}

static void ksu_phi_and_slope(double a, double* phi, double* dphi)
{
    if (a <= 0.0) {
        *phi = 0.0;
        *dphi = 0.0;
        return;
    }
    const double ep = scaled_ei(a), em = -scaled_e1(a);
    const double I = 0.25 * ((a + 1.0) * ep + (a - 1.0) * em);
    const double Ip = 0.25 * (2.0 - a * ep + a * em);
    *phi = 1.0 - 2.0 * I / a;
    *dphi = 2.0 * I / (a * a) - 2.0 * Ip / a;
}

qt_status ensure_ksu_table(qt_context* ctx, int prec, const void** out)
{
    auto it = ctx->ksu_phi.find(prec);
    if (it != ctx->ksu_phi.end()) {
        *out = it->second;
        return QT_OK;
    }
    if (g_no_alloc)
        return fail(QT_EINVAL, "no KSU table on this context yet: run qt_run with it first");
    const int nf = 4097, nc = 16257;
    std::vector<double> v(2 * (size_t)(nf + nc));
    for (int k = 0; k < nf; ++k) ksu_phi_and_slope(k / 8192.0, &v[2 * k], &v[2 * k + 1]);
    for (int k = 0; k < nc; ++k)
        ksu_phi_and_slope(0.5 + k / 256.0, &v[2 * (nf + k)], &v[2 * (nf + k) + 1]);
    void* d = nullptr;
    if (prec == QT_FP32_BULK) {
        std::vector<float> f(v.begin(), v.end());
        QT_HIP(hipMalloc(&d, f.size() * 4));
        QT_HIP(hipMemcpy(d, f.data(), f.size() * 4, hipMemcpyHostToDevice));
    } else {
        QT_HIP(hipMalloc(&d, v.size() * 8));
        QT_HIP(hipMemcpy(d, v.data(), v.size() * 8, hipMemcpyHostToDevice));
    }
    ctx->ksu_phi[prec] = d;
    *out = d;
    return QT_OK;
}

// ------------------------------------------------------ group upload -----

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Highest l with a tabulated static phase.
constexpr int kLTab = 255;


// exp(-i (dt/2) [V_coulomb(r_m) + l(l+1)/(M r_m^2)]) for l = 0..kLTab and
// both colours (appendix "Munich potential"), rows [(2 l + c) N + m]; FP32
// rows hold the factor minus one, (cos - 1, sin), each part rounded once, in
// mirror pairs (mirror_pair_index).
static void phase_table(const HostBatch& h, bool f32, char* dst)
{
    const int N = h.phys.N;
    const double dr = h.phys.L / N, alpha = (4.0 / 3.0) * h.phys.alpha_s;
    for (int l = 0; l <= kLTab; ++l)
        for (int c = 0; c < 2; ++c) {
            const size_t row = (size_t)(2 * l + c) * N;
            const double coul = c == QT_SINGLET ? -alpha : alpha / 8.0;
            const double cent = (double)l * (l + 1) / h.phys.mass;
            for (int m = 0; m < N; ++m) {
                double co = 1.0, sn = 0.0, cm1 = 0.0;
                if (m > 0) {
                    const double r = m * dr;
                    const double th = -0.5 * h.phys.dt * (coul / r + cent / (r * r));
                    co = std::cos(th);
                    sn = std::sin(th);
                    const double sh = std::sin(0.5 * th);
                    cm1 = -2.0 * sh * sh;            // cos th - 1, no cancellation
                }
                if (f32) {
                    // the factor minus one (the kernel applies u + (C - 1) u)
                    float* d = reinterpret_cast<float*>(dst) + 2 * (row + mirror_pair_index(N, m));
                    d[0] = (float)cm1;
                    d[1] = (float)sn;
                } else {
                    double* d = reinterpret_cast<double*>(dst) + 2 * (row + m);
                    d[0] = co;
                    d[1] = sn;
                }
            }
        }
}

qt_status ensure_phase(qt_context* ctx, const HostBatch& h, int prec, const void** out)
{
    std::vector<double> key{(double)prec, (double)h.phys.N, h.phys.L, h.phys.mass, h.phys.alpha_s,
                            h.phys.dt};
    auto it = ctx->phase.find(key);
    if (it != ctx->phase.end()) {
        *out = it->second;
        return QT_OK;
    }
    if (g_no_alloc)
        return fail(QT_EINVAL, "no static phase table for this grid (N, L, mass, alpha_s, dt) "
                    "and precision on this context yet: run qt_run with it first");
    const size_t bytes = (size_t)2 * (kLTab + 1) * h.phys.N * elem_bytes(prec);
    std::vector<char> tab(bytes);
    phase_table(h, prec == QT_FP32_BULK, tab.data());
    void* d = nullptr;
    QT_HIP(hipMalloc(&d, bytes));
    QT_HIP(hipMemcpy(d, tab.data(), bytes, hipMemcpyHostToDevice));
    ctx->phase[key] = d;
    *out = d;
    return QT_OK;
}

qt_status upload_groups(qt_context* ctx, const std::vector<const HostBatch*>& hb, int prec,
                        const std::vector<qt_results>& outs, bool with_Tn, hipStream_t s,
                        bool async_alloc, DeviceGroups* dg, void* into, size_t into_cap)
{
    const bool f32 = prec == QT_FP32_BULK;
    const size_t ng = hb.size();
    size_t off = align_up(ng * sizeof(GroupDesc));
    // the N-sized tables go in once however many groups share them
    struct Offs { size_t tau, T, kin, init, basis, Tn; bool own_kin, own_init, own_basis; };
    std::vector<Offs> o(ng);
    std::map<const void*, size_t> seen;
    auto place = [&](const void* key, size_t bytes, size_t* at) {
        auto it = seen.find(key);
        if (it != seen.end()) {
            *at = it->second;
            return false;
        }
        *at = off;
        off = align_up(off + bytes);
        seen[key] = *at;
        return true;
    };
    for (size_t g = 0; g < ng; ++g) {
        const HostBatch& h = *hb[g];
        const size_t N = h.phys.N;
        o[g].tau = off; off = align_up(off + h.tau.size() * 8);
        o[g].T = off; off = align_up(off + h.T.size() * 8);
        o[g].own_kin = place(h.kin.get(), N * 16, &o[g].kin);
        o[g].own_init = place(h.init.get(), 2 * N * 8, &o[g].init);
        o[g].own_basis = place(h.basis.get(), 6 * N * 8, &o[g].basis);
        o[g].Tn = off;
        if (with_Tn) off = align_up(off + (size_t)std::max<int64_t>(h.n_steps, 1) * 8);
    }
    std::vector<const void*> phase(ng, nullptr), ksu(ng, nullptr);
    if (!with_Tn)
        for (size_t g = 0; g < ng; ++g) {
            qt_status st = ensure_phase(ctx, *hb[g], prec, &phase[g]);
            if (st != QT_OK) return st;
        }
    for (size_t g = 0; g < ng; ++g) {
        if (hb[g]->phys.potential != QT_POTENTIAL_KSU) continue;
        qt_status st = ensure_ksu_table(ctx, prec, &ksu[g]);
        if (st != QT_OK) return st;
    }
    dg->bytes = off;
    if (into) {
        if (off > into_cap)
            return fail(QT_EINVAL, "the batch's tables need %zu bytes, more than the %zu left in "
                        "the static buffer", off, into_cap);
        dg->mem = into;
    } else if (async_alloc) {
        QT_HIP(hipMallocAsync(&dg->mem, off, s));
    } else {
        QT_HIP(hipMalloc(&dg->mem, off));
    }
    char* base = static_cast<char*>(dg->mem);
    std::vector<char> blob(off, 0);
    dg->host.assign(ng, GroupDesc{});
    for (size_t g = 0; g < ng; ++g) {
        const HostBatch& h = *hb[g];
        const int N = h.phys.N;
        GroupDesc d;
        std::memset(&d, 0, sizeof d);
        d.L = h.phys.L; d.dr = h.phys.L / N; d.dt = h.phys.dt; d.mass = h.phys.mass;
        d.alpha = (4.0 / 3.0) * h.phys.alpha_s; d.kappa_hat = h.phys.kappa_hat;
        d.gamma_hat = h.phys.gamma_hat; d.r_max = h.phys.r_max; d.tau_start = h.tau_start;
        d.N = N; d.do_jumps = h.phys.do_jumps; d.max_jumps = h.phys.max_jumps;
        d.init_l = h.init_l; d.init_color = h.init_color; d.flags = h.phys.flags;
        d.n_tab = (int32_t)h.tau.size();
        d.n_steps = h.n_steps; d.n_traj = h.batch.n_traj;
        d.seed = h.batch.seed; d.traj_id0 = h.batch.traj_id0; d.traj_id_stride = h.batch.traj_id_stride;
        d.tau = reinterpret_cast<const double*>(base + o[g].tau);
        d.Ttab = reinterpret_cast<const double*>(base + o[g].T);
        d.kin = base + o[g].kin;
        d.init_psi = reinterpret_cast<const double*>(base + o[g].init);
        d.basis = reinterpret_cast<const double*>(base + o[g].basis);
        d.Tn = with_Tn ? reinterpret_cast<const double*>(base + o[g].Tn) : nullptr;
        d.phase = phase[g];
        d.l_tab = kLTab;
        for (int q = 0; q < 6; ++q) d.init_overlap[q] = h.init->overlap[q];
        d.out = outs[g];
        d.st_psi = nullptr;
        d.st = nullptr;
        d.zeroth = h.zeroth;
        d.zdone = h.zdone;
        d.potential = h.phys.potential;
        d.md_factor = h.phys.md_factor;
        d.ksu_phi = ksu[g];
        dg->host[g] = d;
        std::memcpy(&blob[o[g].tau], h.tau.data(), h.tau.size() * 8);
        std::memcpy(&blob[o[g].T], h.T.data(), h.T.size() * 8);
        if (o[g].own_kin && f32) {
            // in the slot order of the FP32 kinetic block (qt_dst32.hpp):
            // entry n < N/2 is conj(K_k)/4 for the odd output k that the
            // half-length cosine transform leaves in slot n (k = 4n + 1 below
            // N/4, 2N - 4n - 1 above), entry N/2 + q is K_{2q}
            double* k = reinterpret_cast<double*>(&blob[o[g].kin]);
            const int M = N / 2;
            for (int n = 0; n < M; ++n) {
                const int ko = n < M / 2 ? 4 * n + 1 : 2 * N - 4 * n - 1;
                k[2 * n] = 0.25 * (*h.kin)[2 * ko];
                k[2 * n + 1] = -0.25 * (*h.kin)[2 * ko + 1];
                k[2 * (M + n)] = (*h.kin)[4 * n];
                k[2 * (M + n) + 1] = (*h.kin)[4 * n + 1];
            }
        } else if (o[g].own_kin) {
            std::memcpy(&blob[o[g].kin], h.kin->data(), 2 * (size_t)N * 8);
        }
        if (o[g].own_init) std::memcpy(&blob[o[g].init], h.init->psi.data(), 2 * (size_t)N * 8);
        if (o[g].own_basis) std::memcpy(&blob[o[g].basis], h.basis->data(), 6 * (size_t)N * 8);
        if (with_Tn) {
            double* Tn = reinterpret_cast<double*>(&blob[o[g].Tn]);
            for (int64_t n = 0; n < h.n_steps; ++n)
                Tn[n] = host_temperature(h.tau.data(), h.T.data(), (int)h.tau.size(),
                                         h.tau_start + (double)n * h.phys.dt);
        }
    }
    std::memcpy(blob.data(), dg->host.data(), ng * sizeof(GroupDesc));
    dg->groups = reinterpret_cast<GroupDesc*>(base);
    QT_HIP(hipMemcpyAsync(dg->mem, blob.data(), off, hipMemcpyHostToDevice, s));
    // the copy reads pageable memory: wait for it before `blob` goes away
    QT_HIP(hipStreamSynchronize(s));
    return QT_OK;
}

void build_items(const std::vector<const HostBatch*>& hb, std::vector<int32_t>* ig,
                 std::vector<int64_t>* ii)
{
    struct It { double cost; double r; int32_t g; int64_t i; };
    std::vector<It> v;
    size_t total = 0;
    for (const HostBatch* h : hb) total += (size_t)h->batch.n_traj;
    v.reserve(total);
    for (size_t g = 0; g < hb.size(); ++g) {
        const HostBatch& h = *hb[g];
        // a batch's zeroth trajectory goes first: the sooner it finishes, the
        // more of its batch can take its results
        const double cost = (h.phys.flags & kFlagZeroth)
                                ? HUGE_VAL
                                : (double)h.n_steps * h.phys.N * std::log2((double)h.phys.N);
        const bool order_by_r = h.zeroth.norm != nullptr;
        const uint64_t stride = h.batch.traj_id_stride ? h.batch.traj_id_stride : 1u;
        for (int64_t i = 0; i < h.batch.n_traj; ++i) {
            // with the no-jump shortcut, the lowest first thresholds (the
            // trajectories that may take the zeroth's results) go last
            double r = 1.0;
            if (order_by_r)
                r = uniform01(event_block(h.batch.seed, h.batch.traj_id0 + (uint64_t)i * stride, 0).w[2]);
            v.push_back({cost, r, (int32_t)g, i});
        }
    }
    std::stable_sort(v.begin(), v.end(), [](const It& a, const It& b) {
        return a.cost > b.cost || (a.cost == b.cost && a.r > b.r);
    });
    ig->resize(v.size());
    ii->resize(v.size());
    for (size_t k = 0; k < v.size(); ++k) {
        (*ig)[k] = v[k].g;
        (*ii)[k] = v[k].i;
    }
}

// ------------------------------------------------------- variants --------

qt_status choose_variant(qt_context* ctx, int prec, int N, qt_context::Variant* out)
{
    auto key = std::make_pair(prec, N);
    auto it = ctx->plans.find(key);
    if (it != ctx->plans.end()) {
        *out = it->second;
        return QT_OK;
    }
    int Ws[8];
    const int nv = fused_variants(prec, N, Ws, 8);
    if (nv == 0) return fail(QT_EINVAL, "no fused kernel for N=%d precision=%d", N, prec);
    // default (before tuning): 8 complex values per lane when available
    const int want_p = 8;
    int best = Ws[0];
    for (int i = 0; i < nv; ++i)
        if (std::abs(N / Ws[i] - want_p) < std::abs(N / best - want_p)) best = Ws[i];
    qt_context::Variant v;
    v.W = best;
    v.slots_per_cu = fused_occupancy(prec, N, best);
    if (v.slots_per_cu <= 0) return fail(QT_EDEVICE, "kernel N=%d W=%d cannot be resident", N, best);
    ctx->plans[key] = v;
    *out = v;
    return QT_OK;
}

}  // namespace qt

using namespace qt;

// ===================================================================== ABI

extern "C" {

const char* qt_last_error(void) { return g_last_error.c_str(); }
const char* qt_version(void) { return "qtraj-mi355x 0.1 (gfx950)"; }

qt_status qt_context_create(int device, qt_context** out)
{
    if (!out) return fail(QT_EINVAL, "null out");
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n)
        return fail(QT_EDEVICE, "no HIP device %d (%d present)", device, n);
    QT_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    QT_HIP(hipGetDeviceProperties(&prop, device));
    auto* c = new qt_context();
    c->device = device;
    c->n_cu = prop.multiProcessorCount;
    size_t nab = 0;
    if (qt_status st = noalloc_buffer(device, &c->noalloc_buf, &nab); st != QT_OK) {
        delete c;
        return st;
    }
    if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
        delete c;
        return fail(QT_EDEVICE, "hipEventCreate failed");
    }
    *out = c;
    return QT_OK;
}

qt_status qt_context_destroy(qt_context* ctx)
{
    if (!ctx) return QT_OK;
    hipSetDevice(ctx->device);
    hipDeviceSynchronize();
    for (auto& kv : ctx->tables) {
        hipFree(kv.second.tw);
        hipFree(kv.second.prew);
    }
    for (auto& kv : ctx->phase) hipFree(kv.second);
    for (auto& kv : ctx->ksu_phi) hipFree(kv.second);
    for (hipStream_t s : ctx->aux) hipStreamDestroy(s);
    for (hipEvent_t e : ctx->join) hipEventDestroy(e);
    if (ctx->fork) hipEventDestroy(ctx->fork);
    hipEventDestroy(ctx->ev0);
    hipEventDestroy(ctx->ev1);
    delete ctx;
    return QT_OK;
}

qt_status qt_count_steps(const qt_physics* phys, const qt_ttable* ttable, int64_t* n_steps)
{
    if (!phys || !ttable || !n_steps) return fail(QT_EINVAL, "null argument");
    if (!(phys->dt > 0) || !std::isfinite(phys->dt)) return fail(QT_EINVAL, "dt must be finite and > 0");
    if (qt_status st = validate_ttable(ttable); st != QT_OK) return st;
    *n_steps = count_steps(*phys, *ttable);
    return QT_OK;
}

qt_status qt_last_kernel_ms(qt_context* ctx, double* ms, int64_t* launches)
{
    if (!ctx || !ms) return fail(QT_EINVAL, "null argument");
    if (!ctx->timed) return fail(QT_EINVAL, "no timed run on this context");
    QT_HIP(hipSetDevice(ctx->device));
    QT_HIP(hipEventSynchronize(ctx->ev1));
    float f = 0.f;
    QT_HIP(hipEventElapsedTime(&f, ctx->ev0, ctx->ev1));
    *ms = f;
    if (launches) *launches = ctx->last_launches;
    return QT_OK;
}

qt_status qt_plan(qt_context* ctx, int32_t N, int32_t precision, int32_t tune,
                  int32_t* threads_per_traj, int32_t* traj_per_cu);

}  // extern "C"

// -------------------------------------------------------------- runs -----

namespace qt {

qt_status pick_launcher(qt_context* ctx, int prec, int N, int potential, int* W,
                        fused_launcher* launch, int* slots_per_cu)
{
    if (potential == QT_POTENTIAL_KSU) {
        if (!fused_ksu_variant(prec, N, W, launch, slots_per_cu) || *slots_per_cu <= 0)
            return fail(QT_EDEVICE, "no KSU kernel for N=%d", N);
        return QT_OK;
    }
    qt_context::Variant v;
    qt_status st = choose_variant(ctx, prec, N, &v);
    if (st != QT_OK) return st;
    *W = v.W;
    *launch = fused_get(prec, N, v.W);
    *slots_per_cu = v.slots_per_cu;
    return *launch ? QT_OK : fail(QT_EDEVICE, "no kernel for N=%d", N);
}

qt_status run_fused_groups(qt_context* ctx, const std::vector<const HostBatch*>& hb,
                           const std::vector<qt_results>& outs, int prec, hipStream_t s)
{
    // one persistent launch per (grid size N, potential): the kernels are
    // specialised on both; a class is keyed 2 N + potential
    std::vector<int> Ns;
    for (const HostBatch* h : hb) {
        const int key = 2 * h->phys.N + h->phys.potential;
        if (std::find(Ns.begin(), Ns.end(), key) == Ns.end()) Ns.push_back(key);
    }
    DeviceGroups dg;
    qt_status st = upload_groups(ctx, hb, prec, outs, false, s, true, &dg);
    if (st != QT_OK) return st;
    std::vector<int32_t> ig;
    std::vector<int64_t> ii;
    build_items(hb, &ig, &ii);
    // per-N item lists in one allocation: [queues | groups idx | item idx]
    const size_t n_items = ig.size();
    const size_t qbytes = 256;
    const size_t bytes = qbytes + n_items * 4 + 256 + n_items * 8;
    void* mem = nullptr;
    QT_HIP(hipMallocAsync(&mem, bytes, s));
    char* base = static_cast<char*>(mem);
    int32_t* d_ig = reinterpret_cast<int32_t*>(base + qbytes);
    int64_t* d_ii = reinterpret_cast<int64_t*>(base + ((qbytes + n_items * 4 + 255) & ~(size_t)255));
    // reorder items so each N class is contiguous (LPT order kept inside)
    std::vector<int32_t> ig2;
    std::vector<int64_t> ii2;
    std::vector<size_t> start, count;
    for (int key : Ns) {
        start.push_back(ig2.size());
        for (size_t k = 0; k < n_items; ++k)
            if (2 * hb[ig[k]]->phys.N + hb[ig[k]]->phys.potential == key) {
                ig2.push_back(ig[k]);
                ii2.push_back(ii[k]);
            }
        count.push_back(ig2.size() - start.back());
    }
    if (n_items) {
        QT_HIP(hipMemcpyAsync(d_ig, ig2.data(), n_items * 4, hipMemcpyHostToDevice, s));
        QT_HIP(hipMemcpyAsync(d_ii, ii2.data(), n_items * 8, hipMemcpyHostToDevice, s));
        QT_HIP(hipStreamSynchronize(s));
    }
    // The classes run concurrently, each on a stream of its own (the
    // caller's for the first, the context's fork streams, all of default
    // priority, for the others): the workgroups of a class take the CUs that
    // the tail of another class frees instead of waiting for its whole
    // launch to end.  Classes start in the order of their longest item (the
    // items of a class are in LPT order, its first is its longest).
    std::vector<size_t> order;
    for (size_t c = 0; c < Ns.size(); ++c)
        if (count[c] > 0) order.push_back(c);
    auto item_cost = [&](size_t k) {
        const HostBatch& h = *hb[ig2[k]];
        return (double)h.n_steps * h.phys.N * std::log2((double)h.phys.N);
    };
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t x, size_t y) { return item_cost(start[x]) > item_cost(start[y]); });
    std::vector<ClassLaunch> cl;
    for (size_t k = 0; k < order.size(); ++k) {
        const size_t c = order[k];
        const int N = Ns[c] / 2, pot = Ns[c] % 2;
        int W = 0, slots = 0;
        fused_launcher launch = nullptr;
        if ((st = pick_launcher(ctx, prec, N, pot, &W, &launch, &slots)) != QT_OK) return st;
        qt_context::Tables t;
        if ((st = ensure_tables(ctx, prec, N, &t)) != QT_OK) return st;
        FusedArgs a;
        a.groups = dg.groups;
        a.item_group = d_ig + start[c];
        a.item_index = d_ii + start[c];
        a.n_items = (int32_t)count[c];
        a.queue = reinterpret_cast<int32_t*>(base) + c;
        a.tw = t.tw;
        a.prew = t.prew;
        a.seg_steps = 0;
        const int grid = (int)std::min<int64_t>((int64_t)count[c], (int64_t)ctx->n_cu * slots);
        cl.push_back(ClassLaunch{launch, a, grid});
    }
    QT_HIP(hipEventRecord(ctx->ev0, s));
    if ((st = launch_classes(cl, s, &ctx->fork, &ctx->aux, &ctx->join)) != QT_OK) return st;
    const int64_t launches = 2 * (int64_t)cl.size();
    QT_HIP(hipEventRecord(ctx->ev1, s));
    if (trace_on()) {
        QT_HIP(hipEventSynchronize(ctx->ev1));
        float ms = 0.f;
        QT_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        std::string ns;
        for (size_t k = 0; k < order.size(); ++k)
            ns += (k ? "," : "") + std::to_string(Ns[order[k]] / 2);
        trace_line("{\"event\": \"run\", \"precision\": %d, \"batches\": %zu, \"items\": %zu, "
                   "\"N_classes\": [%s], \"kernel_ms\": %.3f}",
                   prec, hb.size(), n_items, ns.c_str(), ms);
    }
    ctx->timed = true;
    ctx->last_launches = launches;
    QT_HIP(hipFreeAsync(mem, s));
    QT_HIP(hipFreeAsync(dg.mem, s));
    return QT_OK;
}

qt_status launch_classes(const std::vector<ClassLaunch>& v, hipStream_t s, hipEvent_t* fork,
                         std::vector<hipStream_t>* streams, std::vector<hipEvent_t>* joins)
{
    if (v.empty()) return QT_OK;
    if (v.size() > 1) {
        if (!*fork) QT_HIP(hipEventCreateWithFlags(fork, hipEventDisableTiming));
        while (streams->size() + 1 < v.size()) {
            hipStream_t a = nullptr;
            hipEvent_t e = nullptr;
            QT_HIP(hipStreamCreateWithFlags(&a, hipStreamNonBlocking));
            streams->push_back(a);
            QT_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            joins->push_back(e);
        }
        QT_HIP(hipEventRecord(*fork, s));
    }
    for (size_t k = 0; k < v.size(); ++k) {
        hipStream_t cs = k == 0 ? s : (*streams)[k - 1];
        if (k > 0) QT_HIP(hipStreamWaitEvent(cs, *fork, 0));
        QT_HIP(launch_queue_reset(v[k].args.queue, cs));
        QT_HIP(v[k].launch(v[k].args, v[k].grid, cs));
    }
    for (size_t k = 1; k < v.size(); ++k) {
        QT_HIP(hipEventRecord((*joins)[k - 1], (*streams)[k - 1]));
        QT_HIP(hipStreamWaitEvent(s, (*joins)[k - 1], 0));
    }
    return QT_OK;
}

// Autotuner: times every compiled variant (threads per trajectory, hence
// radix plan and registers per lane) on a synthetic batch that fills the
// device, and keeps the fastest for (precision, N).
qt_status tune_variant(qt_context* ctx, int prec, int N, qt_context::Variant* out)
{
    int Ws[16];
    const int nv = fused_variants(prec, N, Ws, 16);
    const double tau[2] = {0.0, 1e9}, T[2] = {0.4, 0.4};
    qt_physics p{};
    p.N = N; p.L = N * 5.0 / 256.0; p.dt = 0.001; p.mass = 4.65; p.alpha_s = 0.3;
    p.kappa_hat = 4.0; p.gamma_hat = 0.0; p.deriv_type = 0; p.do_jumps = 1; p.max_jumps = -1;
    p.r_max = 1.0; p.flags = 0;
    qt_ttable tt{tau, T, 2, 0.0, 0.0, 120};
    qt_init in{QT_INIT_GAUSSIAN, 1, 0, QT_SINGLET, 1.0, nullptr, nullptr};
    qt_batch b{};
    b.n_traj = (int64_t)ctx->n_cu * 8; b.seed = 12345; b.traj_id0 = 0; b.traj_id_stride = 1;
    b.precision = prec; b.form = QT_FORM_FUSED;
    HostBatch hb;
    qt_status st = prepare(ctx, &p, &tt, &in, &b, &hb);
    if (st != QT_OK) return st;
    std::vector<const HostBatch*> v{&hb};
    std::vector<qt_results> outs(1);
    std::memset(&outs[0], 0, sizeof(qt_results));
    auto key = std::make_pair(prec, N);
    double best_ms = 1e300;
    qt_context::Variant best{};
    for (int i = 0; i < nv; ++i) {
        qt_context::Variant cand;
        cand.W = Ws[i];
        cand.slots_per_cu = fused_occupancy(prec, N, Ws[i]);
        if (cand.slots_per_cu <= 0) continue;
        ctx->plans[key] = cand;
        double ms = 0;
        for (int rep = 0; rep < 2; ++rep) {   // first run warms up
            if ((st = run_fused_groups(ctx, v, outs, prec, nullptr)) != QT_OK) return st;
            QT_HIP(hipEventSynchronize(ctx->ev1));
            float f = 0.f;
            QT_HIP(hipEventElapsedTime(&f, ctx->ev0, ctx->ev1));
            ms = f;
        }
        if (ms < best_ms) { best_ms = ms; best = cand; }
    }
    if (best.W == 0) return fail(QT_EDEVICE, "no runnable variant for N=%d", N);
    best.tuned = true;
    ctx->plans[key] = best;
    *out = best;
    return QT_OK;
}

qt_status run_plain(qt_context* ctx, const HostBatch& hb, const qt_results& out, hipStream_t s)
{
    const int N = hb.phys.N;
    const int64_t nt = hb.batch.n_traj;
    if (!plain_supported(N)) return fail(QT_EINVAL, "plain form does not support N=%d", N);
    std::vector<const HostBatch*> v{&hb};
    std::vector<qt_results> outs{out};
    DeviceGroups dg;
    qt_status st = upload_groups(ctx, v, QT_FP64, outs, true, s, true, &dg);
    if (st != QT_OK) return st;
    qt_context::Tables t;
    if ((st = ensure_tables(ctx, QT_FP64, N, &t)) != QT_OK) return st;
    double* psi = nullptr;
    TrajState* sts = nullptr;
    QT_HIP(hipMallocAsync(reinterpret_cast<void**>(&psi), std::max<size_t>(1, (size_t)nt * 2 * N * 8), s));
    QT_HIP(hipMallocAsync(reinterpret_cast<void**>(&sts), std::max<size_t>(1, (size_t)nt * sizeof(TrajState)), s));
    PlainArgs a;
    a.g = dg.groups;
    a.psi = psi;
    a.st = sts;
    a.n_traj = nt;
    a.N = N;
    a.tw = t.tw;
    a.prew = t.prew;
    QT_HIP(hipEventRecord(ctx->ev0, s));
    int64_t launches = 0;
    if (nt > 0) {
        QT_HIP(plain_init(a, s));
        launches++;
        for (int64_t n = 0; n < hb.n_steps; ++n) {
            QT_HIP(plain_space(a, n, s));
            QT_HIP(plain_dst(a, s));
            QT_HIP(plain_kinetic(a, s));
            QT_HIP(plain_dst(a, s));
            QT_HIP(plain_space(a, n, s));
            QT_HIP(plain_norm_jump(a, n, s));
            launches += 6;
        }
        QT_HIP(plain_finalize(a, s));
        launches++;
    }
    QT_HIP(hipEventRecord(ctx->ev1, s));
    ctx->timed = true;
    ctx->last_launches = launches;
    QT_HIP(hipFreeAsync(psi, s));
    QT_HIP(hipFreeAsync(sts, s));
    QT_HIP(hipFreeAsync(dg.mem, s));
    return QT_OK;
}

qt_status run_vacuum_phases(qt_context* ctx, const std::vector<HostBatch*>& hb, int prec,
                            hipStream_t s)
{
    // one single-trajectory group per batch with a vacuum phase: T = 0, no
    // jumps, vacuum_steps steps, final state out
    std::vector<HostBatch> vb;
    std::vector<size_t> which, off;
    size_t total = 0;
    for (size_t i = 0; i < hb.size(); ++i) {
        if (hb[i]->vacuum_steps <= 0) continue;
        HostBatch v = *hb[i];
        v.batch.n_traj = 1;
        v.batch.no_jump_shortcut = 0;
        v.phys.do_jumps = 0;
        v.tau = {0.0, 1.0};
        v.T = {0.0, 0.0};
        v.tau_start = 0.0;
        v.n_steps = hb[i]->vacuum_steps;
        v.vacuum_steps = 0;
        v.zeroth = qt_results{};
        vb.push_back(v);
        which.push_back(i);
        off.push_back(total);
        total += 2 * (size_t)v.phys.N;
    }
    if (vb.empty()) return QT_OK;
    double* psi = nullptr;
    QT_HIP(hipMalloc(reinterpret_cast<void**>(&psi), total * sizeof(double)));
    std::vector<const HostBatch*> v;
    std::vector<qt_results> outs(vb.size());
    for (size_t k = 0; k < vb.size(); ++k) {
        v.push_back(&vb[k]);
        std::memset(&outs[k], 0, sizeof(qt_results));
        outs[k].psi = psi + off[k];
    }
    qt_status st = run_fused_groups(ctx, v, outs, prec, s);
    std::vector<double> host(total);
    if (st == QT_OK) {
        hipError_t e = hipMemcpyAsync(host.data(), psi, total * sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = fail(QT_EDEVICE, "vacuum phase: %s", hipGetErrorString(e));
    }
    hipFree(psi);
    if (st != QT_OK) return st;
    for (size_t k = 0; k < vb.size(); ++k) {
        HostBatch& h = *hb[which[k]];
        auto t = std::make_shared<InitTable>();
        t->psi.assign(host.begin() + off[k], host.begin() + off[k] + 2 * (size_t)h.phys.N);
        for (int q = 0; q < 6; ++q) t->overlap[q] = h.init->overlap[q];   // prepared state
        h.init = t;
    }
    return QT_OK;
}

qt_status add_zeroth_groups(const std::vector<HostBatch*>& hb, std::vector<HostBatch>* zb,
                            std::vector<const HostBatch*>* v, std::vector<qt_results>* outs,
                            hipStream_t s, void** mem)
{
    *mem = nullptr;
    size_t nz = 0;
    for (HostBatch* h : hb)
        if (h->batch.no_jump_shortcut && h->phys.do_jumps) ++nz;
    if (nz == 0) return QT_OK;
    // [nz completion flags | per zeroth: 16 doubles (norm, first_r, 6
    // overlaps, 6 survivals, mean_r, min_gap), 4 int32, 1 int64, psi (2N)]
    std::vector<size_t> off;
    size_t total = 256;
    for (HostBatch* h : hb) {
        if (!h->batch.no_jump_shortcut || !h->phys.do_jumps) continue;
        off.push_back(total);
        total += 16 * 8 + 16 + 8 + 2 * (size_t)h->phys.N * 8;
        total = (total + 255) & ~(size_t)255;
    }
    total += ((nz * 4 + 255) & ~(size_t)255);
    char* base = nullptr;
    QT_HIP(hipMallocAsync(reinterpret_cast<void**>(&base), total, s));
    int32_t* flags = reinterpret_cast<int32_t*>(base + total - ((nz * 4 + 255) & ~(size_t)255));
    QT_HIP(launch_zero_i32(flags, (int64_t)nz, s));
    zb->reserve(nz);
    size_t k = 0;
    for (HostBatch* h : hb) {
        if (!h->batch.no_jump_shortcut || !h->phys.do_jumps) continue;
        double* d = reinterpret_cast<double*>(base + off[k]);
        int32_t* i4 = reinterpret_cast<int32_t*>(d + 16);
        qt_results r{};
        r.norm = d; r.first_r = d + 1; r.overlap = d + 2; r.survival = d + 8;
        r.mean_r = d + 14; r.min_gap = d + 15;
        r.l = i4; r.color = i4 + 1; r.n_jumps = i4 + 2; r.status = i4 + 3;
        r.steps_done = reinterpret_cast<int64_t*>(i4 + 4);
        r.psi = reinterpret_cast<double*>(i4 + 6);
        HostBatch z = *h;
        z.batch.n_traj = 1;
        z.batch.no_jump_shortcut = 0;
        z.phys.flags |= kFlagZeroth;
        z.zeroth = qt_results{};
        z.zdone = flags + k;
        zb->push_back(z);
        v->push_back(&zb->back());
        outs->push_back(r);
        h->zeroth = r;
        h->zdone = flags + k;
        ++k;
    }
    *mem = base;
    return QT_OK;
}

}  // namespace qt

extern "C" {

qt_status qt_run(qt_context* ctx, const qt_physics* phys, const qt_ttable* tt, const qt_init* init,
                 const qt_batch* batch, const qt_results* dev_out, void* hip_stream)
{
    if (!ctx || !dev_out) return fail(QT_EINVAL, "null argument");
    if (dev_out->jump_log_cap < 0) return fail(QT_EINVAL, "jump_log_cap < 0");
    std::lock_guard<std::mutex> lk(ctx->mu);
    QT_HIP(hipSetDevice(ctx->device));
    HostBatch hb;
    qt_status st = prepare(ctx, phys, tt, init, batch, &hb);
    if (st != QT_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    std::vector<HostBatch*> hv{&hb};
    if ((st = run_vacuum_phases(ctx, hv, batch->precision, s)) != QT_OK) return st;
    if (batch->form == QT_FORM_PLAIN) return run_plain(ctx, hb, *dev_out, s);
    std::vector<const HostBatch*> v{&hb};
    std::vector<qt_results> outs{*dev_out};
    std::vector<HostBatch> zb;
    void* zmem = nullptr;
    if ((st = add_zeroth_groups(hv, &zb, &v, &outs, s, &zmem)) != QT_OK) return st;
    st = run_fused_groups(ctx, v, outs, batch->precision, s);
    if (zmem) hipFreeAsync(zmem, s);
    return st;
}

qt_status qt_run_many(qt_context* ctx, int32_t n_batches, const qt_physics* phys,
                      const qt_ttable* tt, const qt_init* init, const qt_batch* batch,
                      const qt_results* dev_out, void* hip_stream)
{
    if (!ctx || n_batches < 1 || !phys || !tt || !init || !batch || !dev_out)
        return fail(QT_EINVAL, "null argument or no batches");
    std::lock_guard<std::mutex> lk(ctx->mu);
    QT_HIP(hipSetDevice(ctx->device));
    std::vector<HostBatch> hbs(n_batches);
    for (int i = 0; i < n_batches; ++i) {
        if (dev_out[i].jump_log_cap < 0) return fail(QT_EINVAL, "batch %d: jump_log_cap < 0", i);
        qt_status st = prepare(ctx, &phys[i], &tt[i], &init[i], &batch[i], &hbs[i]);
        if (st != QT_OK) return fail(st, "batch %d: %s", i, g_last_error.c_str());
        if (batch[i].form != QT_FORM_FUSED) return fail(QT_EINVAL, "batch %d: qt_run_many runs the fused form", i);
        if (batch[i].precision != batch[0].precision) return fail(QT_EINVAL, "batch %d: mixed precision", i);
    }
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    std::vector<HostBatch*> hv;
    for (auto& h : hbs) hv.push_back(&h);
    qt_status st = run_vacuum_phases(ctx, hv, batch[0].precision, s);
    if (st != QT_OK) return st;
    std::vector<const HostBatch*> v;
    std::vector<qt_results> outs;
    for (int i = 0; i < n_batches; ++i) {
        v.push_back(&hbs[i]);
        outs.push_back(dev_out[i]);
    }
    std::vector<HostBatch> zb;
    void* zmem = nullptr;
    if ((st = add_zeroth_groups(hv, &zb, &v, &outs, s, &zmem)) != QT_OK) return st;
    st = run_fused_groups(ctx, v, outs, batch[0].precision, s);
    if (zmem) hipFreeAsync(zmem, s);
    return st;
}

qt_status qt_plan_variants(int32_t N, int32_t precision, int32_t* threads, int32_t cap,
                           int32_t* count)
{
    if (!count || cap < 0 || (cap > 0 && !threads)) return fail(QT_EINVAL, "null argument or negative cap");
    int Ws[16];
    const int n = fused_variants(precision, N, Ws, 16);
    std::sort(Ws, Ws + n);
    for (int i = 0; i < n && i < cap; ++i) threads[i] = Ws[i];
    *count = n;
    return QT_OK;
}

qt_status qt_plan_set(qt_context* ctx, int32_t N, int32_t precision, int32_t threads_per_traj)
{
    if (!ctx) return fail(QT_EINVAL, "null context");
    if (!fused_get(precision, N, threads_per_traj))
        return fail(QT_EINVAL, "no fused kernel for N=%d precision=%d with %d threads per trajectory",
                    N, precision, threads_per_traj);
    std::lock_guard<std::mutex> lk(ctx->mu);
    QT_HIP(hipSetDevice(ctx->device));
    qt_context::Variant v;
    v.W = threads_per_traj;
    v.slots_per_cu = fused_occupancy(precision, N, threads_per_traj);
    v.tuned = true;
    if (v.slots_per_cu <= 0)
        return fail(QT_EDEVICE, "kernel N=%d W=%d cannot be resident", N, threads_per_traj);
    ctx->plans[std::make_pair(precision, N)] = v;
    return QT_OK;
}

qt_status qt_plan(qt_context* ctx, int32_t N, int32_t precision, int32_t tune,
                  int32_t* threads_per_traj, int32_t* traj_per_cu)
{
    if (!ctx) return fail(QT_EINVAL, "null context");
    std::lock_guard<std::mutex> lk(ctx->mu);
    QT_HIP(hipSetDevice(ctx->device));
    qt_context::Variant v;
    qt_status st = choose_variant(ctx, precision, N, &v);
    if (st != QT_OK) return st;
    if (tune && !v.tuned) {
        if ((st = tune_variant(ctx, precision, N, &v)) != QT_OK) return st;
    }
    if (threads_per_traj) *threads_per_traj = v.W;
    if (traj_per_cu) *traj_per_cu = v.slots_per_cu;
    return QT_OK;
}

}  // extern "C"
