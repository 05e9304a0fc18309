/*
 * qtraj_oracle.c -- CPU FP64 reference for the quantum-trajectory solver of
 * QTraj 1.0 (Ba Omar, Escobedo, Islam, Strickland, Thapa, Vander Griend,
 * Weber; arXiv:2107.06147).
 *
 * TEST INFRASTRUCTURE ONLY: the plain, slow, obviously correct statement of
 * the method that the GPU library is checked against.  Nothing here is
 * blocked, fused or reordered: every step is taken in the order the paper
 * gives, with an O(N^2) sine transform written straight from its definition.
 * It shares no code with the GPU library.
 *
 * Paper passages followed (section titles and equation labels of the paper):
 *   - Sec. "Algorithm for deterministic evolution between quantum jumps":
 *     eq. (uUpdate), the five-step Strang split, eq. (normcond), the sine
 *     series that enforces u(0)=0.
 *   - Sec. "Derivative types": T_kin = p^2/m with m the heavy-quark mass,
 *     or T_discrete = 2[1-cos(p dr)]/(m dr^2).
 *   - Appendix "Munich potential": singlet/octet real and imaginary parts,
 *     alpha = C_F alpha_s, kappa = kappa_hat T^3, gamma = gamma_hat T^3, and
 *     the centrifugal term l(l+1)/(m r^2) of the radial problem.
 *   - Sec. "The waiting time approach": evolve until the norm is <= r, jump,
 *     renormalise, draw a new r.
 *   - Sec. "Summary of QTraj execution", step 4: rMax and maxJumps handling,
 *     l then colour update, multiplication by r.
 *   - Eqs. (Pl+-) and (pjump) and the colour probabilities p_{o->s} = 2/7,
 *     p_{s->o} = 1.
 *   - Eq. (hamiltonian)/(hsoCoul): Coulomb basis states with Bohr radius
 *     a0 = 2/(m alpha) (reduced mass m/2).
 *
 * Readings of points the paper leaves open (each is a stated choice):
 *   - grid: r_j = j L/N, j = 1..N-1, u(L) = 0; DST-I of the N-1 interior
 *     points, p_k = pi k / L;
 *   - T between table points: linear in tau; both half-steps of step n use
 *     T(t_n), t_n = tau_start + n dt;
 *   - a jump happens iff norm <= r, also on the last step;
 *   - maxJumps: when the norm reaches r and nJumps == maxJumps the trajectory
 *     ends with zero overlaps;
 *   - r > rMax: zero overlaps, no evolution;
 *   - overlaps use the normalised final state |<b|u>|^2 / <u|u>;
 *     survival = overlap / initial overlap when the initial overlap is
 *     non-zero, else the raw overlap;
 *   - Gaussian initial state u ~ r^{l+1} exp(-r^2 / (2 width^2));
 *   - random numbers: Philox4x64-10 (Salmon et al., SC'11), key (seed, 0),
 *     counter (event+1, trajectory id, 0, 0); event 0 is the start, event e
 *     the e-th jump; words 0, 1, 2 give u_l, u_c and the next threshold,
 *     u = ((w >> 12) + 0.5) 2^-52, strictly inside (0,1).
 */
#include "qtraj_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Random numbers: Philox4x64-10 from its published definition.              */
/* ------------------------------------------------------------------------ */
void qto_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        unsigned __int128 p0 = (unsigned __int128)M0 * x0;
        unsigned __int128 p1 = (unsigned __int128)M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += W0; k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

double qto_uniform(uint64_t word)
{
    /* open interval (0,1): the top 52 bits plus one half, scaled by 2^-52;
     * every value is exact, the largest is 1 - 2^-53 < 1 */
    return ((double)(word >> 12) + 0.5) * (1.0 / 4503599627370496.0);
}

static void event_block(uint64_t seed, uint64_t traj_id, int64_t event, uint64_t w[4])
{
    uint64_t ctr[4] = { (uint64_t)event + 1u, traj_id, 0u, 0u };
    uint64_t key[2] = { seed, 0u };
    qto_philox4x64_10(ctr, key, w);
}

/* ------------------------------------------------------------------------ */
/* Jump rule: eqs. (Pl+-), (pjump); colour probabilities.                   */
/* ------------------------------------------------------------------------ */
static void apply_jump_rule(double u_l, double u_c, int32_t* l, int32_t* c)
{
    /* angular momentum first: down with probability l/(2l+1) */
    double p_down = (double)(*l) / (double)(2 * (*l) + 1);
    if (u_l < p_down) *l = *l - 1;
    else              *l = *l + 1;
    /* colour: singlet -> octet always; octet -> singlet with 2/7 */
    if (*c == QTO_OCTET) {
        if (u_c < 2.0 / 7.0) *c = QTO_SINGLET;
        else                 *c = QTO_OCTET;
    } else {
        *c = QTO_OCTET;
    }
}

void qto_jump_rule(uint64_t seed, uint64_t traj_id, int64_t event,
                   int32_t l, int32_t c, int32_t* l_new, int32_t* c_new)
{
    uint64_t w[4];
    event_block(seed, traj_id, event, w);
    apply_jump_rule(qto_uniform(w[0]), qto_uniform(w[1]), &l, &c);
    *l_new = l;
    *c_new = c;
}

/* ------------------------------------------------------------------------ */
/* Temperature table: linear interpolation in tau, clamped at the ends.     */
/* ------------------------------------------------------------------------ */
double qto_temperature(const qto_ttable* tt, double t)
{
    int32_t n = tt->n;
    if (t <= tt->tau[0]) return tt->T[0];
    if (t >= tt->tau[n - 1]) return tt->T[n - 1];
    int32_t i = 0;
    while (!(tt->tau[i + 1] > t)) ++i;   /* tau[i] <= t < tau[i+1] */
    double w = (t - tt->tau[i]) / (tt->tau[i + 1] - tt->tau[i]);
    return tt->T[i] + (tt->T[i + 1] - tt->T[i]) * w;
}

int64_t qto_num_steps(const qto_physics* p, const qto_ttable* tt)
{
    int64_t n = 0;
    while (n < tt->max_steps) {
        double t = tt->tau_start + (double)n * p->dt;
        if (t > tt->tau[tt->n - 1]) break;
        if (qto_temperature(tt, t) < tt->T_final) break;
        ++n;
    }
    return n;
}

/* ------------------------------------------------------------------------ */
/* DST-I straight from its definition, O(N^2).                              */
/* ------------------------------------------------------------------------ */
static double* sine_table(int32_t N)
{
    /* sin(pi m / N) for m = 0..2N-1; sin(pi j k / N) = tab[(j k) mod 2N] */
    double* tab = (double*)malloc(sizeof(double) * 2 * (size_t)N);
    for (int32_t m = 0; m < 2 * N; ++m) tab[m] = sin(PI * (double)m / (double)N);
    return tab;
}

static void dst1_with_table(int32_t N, const double* tab, const double* in_re,
                            const double* in_im, double* out_re, double* out_im)
{
    double scale = sqrt(2.0 / (double)N);
    out_re[0] = 0.0;
    out_im[0] = 0.0;
    for (int32_t k = 1; k < N; ++k) {
        double sr = 0.0, si = 0.0;
        int32_t jk = 0;               /* (j k) mod 2N, stepped by k */
        for (int32_t j = 1; j < N; ++j) {
            jk += k;
            if (jk >= 2 * N) jk -= 2 * N;
            double s = tab[jk];
            sr += in_re[j] * s;
            si += in_im[j] * s;
        }
        out_re[k] = scale * sr;
        out_im[k] = scale * si;
    }
}

void qto_dst1(int32_t N, const double* in_re, const double* in_im,
              double* out_re, double* out_im)
{
    double* tab = sine_table(N);
    dst1_with_table(N, tab, in_re, in_im, out_re, out_im);
    free(tab);
}

/* ------------------------------------------------------------------------ */
/* Physics pieces.                                                          */
/* ------------------------------------------------------------------------ */
static double coulomb_alpha(const qto_physics* p) { return (4.0 / 3.0) * p->alpha_s; }

/* Kinetic energy of mode k (Sec. "Derivative types"). */
static double kinetic_energy(const qto_physics* p, int32_t k)
{
    double dr = p->L / (double)p->N;
    double pk = PI * (double)k / p->L;
    if (p->deriv_type == 1) return 2.0 * (1.0 - cos(pk * dr)) / (p->mass * dr * dr);
    return pk * pk / p->mass;
}

/* kappa_hat at temperature T: the constant kappa_hat >= 0, or one of the
 * fits to lattice data (appendix "Munich potential", the kappa_hat(T)
 * parameterisation): kappa_hat = 1 / (a x^{3/2} + b x + c x^{1/2} + d),
 * x = T / T_c, T_c = 155 MeV, for kappa_hat = -1 (central), -2 (lower),
 * -3 (upper fit).  Below the fits' range, where the denominator is not
 * positive (T below about 0.3 T_c), kappa_hat is taken as 0. */
double qto_kappa_hat(double kappa_hat, double T)
{
    static const double fit[3][4] = {
        { 0.00397, -0.08341, 0.98031, -0.51889 },   /* central */
        { 0.00712, -0.14262, 1.55601, -0.80712 },   /* lower   */
        { 0.00272, -0.05854, 0.71513, -0.38197 },   /* upper   */
    };
    if (kappa_hat >= 0.0) return kappa_hat;
    int k = (int)(-kappa_hat) - 1;
    double x = T / 0.155;
    double sx = sqrt(x);
    double den = fit[k][0] * x * sx + fit[k][1] * x + fit[k][2] * sx + fit[k][3];
    return den > 0.0 ? 1.0 / den : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Isotropic KSU potential (appendix "Isotropic KSU potential").            */
/* ------------------------------------------------------------------------ */

/* Ei(x) for x > 0: gamma + ln x + sum_k x^k / (k k!) (all terms positive). */
static double ei_pos(double x)
{
    double term = 1.0, sum = 0.0;
    for (int k = 1; k < 1000; ++k) {
        term *= x / (double)k;
        double add = term / (double)k;
        sum += add;
        if (add < 1e-17 * sum) break;
    }
    return 0.57721566490153286061 + log(x) + sum;
}

/* exp(x) E1(x), x > 0: the series E1 = -gamma - ln x - sum (-x)^k/(k k!) for
 * x <= 1, the continued fraction E1 = exp(-x) / (x + 1 - 1/(x + 3 - 4/(x + 5
 * - ...))) evaluated backwards from a deep truncation for x > 1. */
static double exp_e1(double x)
{
    if (x <= 1.0) {
        double term = 1.0, sum = 0.0;
        for (int k = 1; k < 60; ++k) {
            term *= -x / (double)k;
            sum += term / (double)k;
        }
        return exp(x) * (-0.57721566490153286061 - log(x) - sum);
    }
    double f = 0.0;
    for (int k = 400; k >= 1; --k) f = (double)k * (double)k / (x + 2.0 * k + 1.0 - f);
    return 1.0 / (x + 1.0 - f);
}

/* phi(a) = 2 int_0^inf dz z/(z^2+1)^2 [1 - sin(z a)/(z a)]
 *        = 1 - (2/a) I(a),  I(a) = int_0^inf sin(a z)/(1+z^2)^2 dz
 *        = [(a+1) e^{-a} Ei(a) + (a-1) e^{a} Ei(-a)] / 4,
 * the closed form from the sine integral of 1/(z^2+b^2) in terms of Ei,
 * differentiated in b at b = 1.  For large a the asymptotic series
 * 1 - 2/a^2 - 8/a^4 - 144/a^6 - 5760/a^8 - 403200/a^10 (from the
 * derivatives of 1/(1+z^2)^2 at 0). */
double qto_ksu_phi(double a)
{
    if (a <= 0.0) return 0.0;
    if (a >= 100.0) {
        double q = 1.0 / (a * a);
        return 1.0 - q * (2.0 + q * (8.0 + q * (144.0 + q * (5760.0 + q * 403200.0))));
    }
    double ep = exp(-a) * ei_pos(a);          /* e^{-a} Ei(a)  */
    double em = -exp_e1(a);                   /* e^{a} Ei(-a)  */
    double I = 0.25 * ((a + 1.0) * ep + (a - 1.0) * em);
    return 1.0 - 2.0 * I / a;
}

/* Constants of the KSU potential: effective coupling, string tension,
 * string-breaking distance 1.25 fm, alpha_s(5 GeV) = 0.2034 run at one loop
 * with N_F = 3 light flavours (b0 = 11 - 2 N_F/3) to the scale 2 pi T. */
static const double KSU_A = 0.409, KSU_SIGMA = 0.21, KSU_RSB = 1.25 / 0.1973269804;
static const double KSU_AS0 = 0.2034, KSU_MU0 = 5.0, KSU_NF = 3.0, KSU_NC = 3.0;

/* alpha_s(2 pi T); <= 0 at and below the one-loop pole (no medium there). */
static double ksu_alpha_s(double T)
{
    if (!(T > 0.0)) return 0.0;
    double inv = 1.0 / KSU_AS0 + (11.0 - 2.0 * KSU_NF / 3.0) / (2.0 * PI) * log(2.0 * PI * T / KSU_MU0);
    return inv > 0.0 ? 1.0 / inv : 0.0;
}

static void ksu_potential(const qto_physics* p, double r, int32_t l, double T, double* VR, double* VI)
{
    double as = ksu_alpha_s(T);
    double mD = 0.0;
    if (as > 0.0)
        mD = p->md_factor * T * sqrt(KSU_NC * (1.0 + KSU_NF / 6.0) * PI * (4.0 / 3.0) * as);
    double x = mD * r;
    /* (1 - e^{-x})/x, 1 at x = 0 */
    double q = x > 0.0 ? -expm1(-x) / x : 1.0;
    double e = exp(-x);
    double kms = -KSU_A / r * (1.0 + x) * e + 2.0 * KSU_SIGMA * r * q - KSU_SIGMA * r * e;
    double vsb = -KSU_A / KSU_RSB + KSU_SIGMA * KSU_RSB;
    *VR = (kms <= vsb ? kms : vsb) + (double)l * (double)(l + 1) / (p->mass * r * r);
    *VI = -as * (4.0 / 3.0) * T * qto_ksu_phi(x);
}

/* V_eff = V_R + i V_I of the Munich potential plus the centrifugal term. */
static void munich_potential(const qto_physics* p, double r, int32_t l, int32_t c,
                             double T, double* VR, double* VI)
{
    if (p->potential == QTO_POTENTIAL_KSU) {
        ksu_potential(p, r, l, T, VR, VI);
        return;
    }
    double alpha = coulomb_alpha(p);
    double kappa = qto_kappa_hat(p->kappa_hat, T) * T * T * T;
    double gamma = p->gamma_hat * T * T * T;
    double centrifugal = (double)l * (double)(l + 1) / (p->mass * r * r);
    if (c == QTO_SINGLET) {
        *VR = -alpha / r + 0.5 * gamma * r * r + centrifugal;
        *VI = -0.5 * kappa * r * r;
    } else {
        *VR = alpha / (8.0 * r) + (7.0 / 32.0) * gamma * r * r + centrifugal;
        *VI = -(7.0 / 32.0) * kappa * r * r;
    }
}

/* Hydrogen-like radial function u = r R_nl with Bohr radius a0. */
/* The potential V_R + i V_I at r for angular momentum l and colour c at
 * temperature T, and the kinetic energy of sine mode k: the two parts of
 * the Hamiltonian, exported for the vacuum eigenstates (Sec. "Using the
 * built-in eigensolvers"). */
void qto_potential(const qto_physics* p, double r, int32_t l, int32_t c, double T,
                   double* VR, double* VI)
{
    munich_potential(p, r, l, c, T, VR, VI);
}

double qto_kinetic_energy(const qto_physics* p, int32_t k) { return kinetic_energy(p, k); }

static double hydrogen_u(int32_t n, int32_t l, double a0, double r)
{
    double x = r / a0;
    if (n == 1 && l == 0) return 2.0 * pow(a0, -1.5) * r * exp(-x);
    if (n == 2 && l == 0) return (1.0 / sqrt(2.0)) * pow(a0, -1.5) * r * (1.0 - x / 2.0) * exp(-x / 2.0);
    if (n == 2 && l == 1) return (1.0 / (2.0 * sqrt(6.0))) * pow(a0, -2.5) * r * r * exp(-x / 2.0);
    if (n == 3 && l == 0) return (2.0 / (3.0 * sqrt(3.0))) * pow(a0, -1.5) * r
                               * (1.0 - 2.0 * x / 3.0 + 2.0 * x * x / 27.0) * exp(-x / 3.0);
    if (n == 3 && l == 1) return (8.0 / (27.0 * sqrt(6.0))) * pow(a0, -2.5) * r * r
                               * (1.0 - x / 6.0) * exp(-x / 3.0);
    if (n == 3 && l == 2) return (4.0 / (81.0 * sqrt(30.0))) * pow(a0, -3.5) * r * r * r * exp(-x / 3.0);
    return NAN;
}

static const int32_t BASIS_N[6] = { 1, 2, 2, 3, 3, 3 };
static const int32_t BASIS_L[6] = { 0, 0, 1, 0, 1, 2 };

/* Normalise a real vector with eq. (normcond). */
static void normalise_real(int32_t N, double dr, double* u)
{
    double s = 0.0;
    for (int32_t j = 1; j < N; ++j) s += u[j] * u[j];
    double f = 1.0 / sqrt(dr * s);
    for (int32_t j = 0; j < N; ++j) u[j] *= f;
}

int qto_basis_state(int32_t N, double L, double mass, double alpha_s,
                    int32_t n, int32_t l, double* u)
{
    double dr = L / (double)N;
    double a0 = 2.0 / (mass * (4.0 / 3.0) * alpha_s);
    u[0] = 0.0;
    for (int32_t j = 1; j < N; ++j) u[j] = hydrogen_u(n, l, a0, (double)j * dr);
    if (isnan(u[1])) return -1;
    normalise_real(N, dr, u);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Per-trajectory work space.                                               */
/* ------------------------------------------------------------------------ */
typedef struct {
    double* re; double* im;       /* u_j                                     */
    double* tre; double* tim;     /* the state in sine-mode space            */
    double* fre; double* fim;     /* half-step factor exp(-i V_eff dt/2)     */
} workspace;

static double norm_of(int32_t N, double dr, const double* re, const double* im)
{
    double s = 0.0;
    for (int32_t j = 1; j < N; ++j) s += re[j] * re[j] + im[j] * im[j];
    return dr * s;
}

/* The position-space factor of eq. (uUpdate), exp(-i V_eff dt/2) with
 * V_eff = V_R + i V_I, at every grid point: its modulus exp(V_I dt/2) and
 * its phase -V_R dt/2. */
static void half_step_factor(const qto_physics* p, int32_t l, int32_t c, double T, workspace* w)
{
    double dr = p->L / (double)p->N;
    w->fre[0] = 0.0; w->fim[0] = 0.0;
    for (int32_t j = 1; j < p->N; ++j) {
        double VR, VI;
        munich_potential(p, (double)j * dr, l, c, T, &VR, &VI);
        double modulus = exp(0.5 * p->dt * VI);
        double angle = -0.5 * p->dt * VR;
        w->fre[j] = modulus * cos(angle);
        w->fim[j] = modulus * sin(angle);
    }
}

/* a_j <- a_j f_j for complex a and f */
static void pointwise_mul(int32_t N, double* are, double* aim, const double* fre, const double* fim)
{
    for (int32_t j = 0; j < N; ++j) {
        double x = are[j], y = aim[j];
        are[j] = x * fre[j] - y * fim[j];
        aim[j] = x * fim[j] + y * fre[j];
    }
}

/* One time step, eq. (uUpdate): u <- F S E S F u, with F the half-step
 * factor (w->f), S the sine transform of the grid (on the real and the
 * imaginary part alike) and E = diag(exp(-i E_k dt)) the kinetic factor in
 * sine-mode space.  S is applied out of place, from u into t and back. */
static void strang_step(int32_t N, const double* sines, workspace* w,
                        const double* ere, const double* eim)
{
    pointwise_mul(N, w->re, w->im, w->fre, w->fim);
    dst1_with_table(N, sines, w->re, w->im, w->tre, w->tim);
    pointwise_mul(N, w->tre, w->tim, ere, eim);
    dst1_with_table(N, sines, w->tre, w->tim, w->re, w->im);
    pointwise_mul(N, w->re, w->im, w->fre, w->fim);
}

/* Singlet overlaps |<b|u>|^2 / <u|u> for the six basis states. */
static void singlet_overlaps(int32_t N, double dr, const double* basis, int32_t l, int32_t c,
                             const double* re, const double* im, double out[6])
{
    double nrm = norm_of(N, dr, re, im);
    for (int b = 0; b < 6; ++b) {
        if (c != QTO_SINGLET || l != BASIS_L[b] || !(nrm > 0.0)) { out[b] = 0.0; continue; }
        const double* phi = basis + (size_t)b * N;
        double ar = 0.0, ai = 0.0;
        for (int32_t j = 1; j < N; ++j) { ar += phi[j] * re[j]; ai += phi[j] * im[j]; }
        ar *= dr; ai *= dr;
        out[b] = (ar * ar + ai * ai) / nrm;
    }
}

static double mean_radius(int32_t N, double dr, const double* re, const double* im)
{
    double num = 0.0, den = 0.0;
    for (int32_t j = 1; j < N; ++j) {
        double w2 = re[j] * re[j] + im[j] * im[j];
        num += (double)j * dr * w2;
        den += w2;
    }
    return den > 0.0 ? num / den : 0.0;
}

/* Initial state (Sec. "Code parameters", initType; Coulomb or Gaussian). */
static int initial_state(const qto_physics* p, const qto_init* ini, double* re, double* im)
{
    int32_t N = p->N;
    double dr = p->L / (double)N;
    re[0] = 0.0; im[0] = 0.0;
    if (ini->kind == QTO_INIT_COULOMB) {
        if (qto_basis_state(N, p->L, p->mass, p->alpha_s, ini->n, ini->l, re) != 0) return -1;
        for (int32_t j = 0; j < N; ++j) im[j] = 0.0;
        return 0;
    }
    if (ini->kind == QTO_INIT_GAUSSIAN) {
        for (int32_t j = 1; j < N; ++j) {
            double r = (double)j * dr;
            re[j] = pow(r, (double)(ini->l + 1)) * exp(-r * r / (2.0 * ini->width * ini->width));
            im[j] = 0.0;
        }
    } else if (ini->kind == QTO_INIT_ARRAY) {
        for (int32_t j = 1; j < N; ++j) { re[j] = ini->u_re[j]; im[j] = ini->u_im ? ini->u_im[j] : 0.0; }
    } else {
        return -1;
    }
    double nrm = norm_of(N, dr, re, im);
    if (!(nrm > 0.0)) return -1;
    double f = 1.0 / sqrt(nrm);
    for (int32_t j = 1; j < N; ++j) { re[j] *= f; im[j] *= f; }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The trajectory loop (Secs. "The waiting time approach" and "Summary of   */
/* QTraj execution", step 4).                                               */
/* ------------------------------------------------------------------------ */
typedef struct {
    const qto_physics* p; const qto_ttable* tt; const qto_init* ini; const qto_batch* b;
    qto_results* out; int64_t n_steps;
    const double* tab; const double* mom_re; const double* mom_im;
    const double* basis; const double* init_re; const double* init_im;
    double init_overlap[6];
    /* the zeroth trajectory (no_jump_shortcut): its smallest norm over the
       run, and its results in `zeroth` (one entry, with its norm trace) */
    int have_zeroth;
    double r_min;
    const qto_results* zeroth;
} shared_setup;

/* Copies entry 0 of the zeroth trajectory's results to entry i: a trajectory
 * whose first threshold r lies below every norm of the no-jump evolution
 * never jumps, so its evolution is that evolution (Sec. "Summary of QTraj
 * execution", step 4: r_0 < rMin = p_NoJumps).  Only first_r, the gap and
 * the status are its own. */
static void take_zeroth(const shared_setup* s, int64_t i, double r)
{
    const qto_results* z = s->zeroth;
    qto_results* out = s->out;
    int32_t N = s->p->N;
    if (out->norm) out->norm[i] = z->norm[0];
    if (out->first_r) out->first_r[i] = r;
    if (out->overlap) for (int bb = 0; bb < 6; ++bb) out->overlap[6 * i + bb] = z->overlap[bb];
    if (out->survival) for (int bb = 0; bb < 6; ++bb) out->survival[6 * i + bb] = z->survival[bb];
    if (out->mean_r) out->mean_r[i] = z->mean_r[0];
    if (out->l) out->l[i] = z->l[0];
    if (out->color) out->color[i] = z->color[0];
    if (out->n_jumps) out->n_jumps[i] = 0;
    if (out->status) out->status[i] = QTO_STATUS_NOJUMP;
    if (out->steps_done) out->steps_done[i] = z->steps_done[0];
    if (out->min_gap) out->min_gap[i] = s->r_min - r;
    if (out->psi) memcpy(out->psi + (size_t)i * 2 * N, z->psi, sizeof(double) * 2 * N);
    if (out->norm_trace)
        memcpy(out->norm_trace + i * s->n_steps, z->norm_trace, sizeof(double) * s->n_steps);
}

/* zeroth != 0: the zeroth trajectory, whose threshold is 0 so that it never
 * jumps; its gap min |norm - 0| is then its smallest norm. */
static void run_one(const shared_setup* s, int64_t i, workspace* w, int zeroth)
{
    const qto_physics* p = s->p;
    int32_t N = p->N;
    double dr = p->L / (double)N;
    uint64_t stride = s->b->traj_id_stride ? s->b->traj_id_stride : 1u;
    uint64_t traj_id = s->b->traj_id0 + (uint64_t)i * stride;
    qto_results* out = s->out;

    memcpy(w->re, s->init_re, sizeof(double) * N);
    memcpy(w->im, s->init_im, sizeof(double) * N);
    int32_t l = s->ini->l, c = s->ini->color, n_jumps = 0, status = QTO_STATUS_OK;
    int64_t steps = 0;
    double min_gap = INFINITY;
    int32_t logged = 0;

    /* the first threshold r_0 */
    uint64_t wd[4];
    event_block(s->b->seed, traj_id, 0, wd);
    double r = zeroth ? 0.0 : qto_uniform(wd[2]);
    double first_r = r;
    double norm = norm_of(N, dr, w->re, w->im);

    if (!zeroth && s->have_zeroth && r < s->r_min) {
        take_zeroth(s, i, r);
        return;
    }
    if (p->do_jumps && r > p->r_max) {
        status = QTO_STATUS_RMAX;
    } else {
        for (int64_t n = 0; n < s->n_steps; ++n) {
            double T = qto_temperature(s->tt, s->tt->tau_start + (double)n * p->dt);
            half_step_factor(p, l, c, T, w);
            strang_step(N, s->tab, w, s->mom_re, s->mom_im);
            norm = norm_of(N, dr, w->re, w->im);
            steps = n + 1;
            if (out->norm_trace) out->norm_trace[i * s->n_steps + n] = norm;
            if (!p->do_jumps) continue;
            double gap = fabs(norm - r);
            if (gap < min_gap) min_gap = gap;
            if (norm <= r) {
                if (p->max_jumps >= 0 && n_jumps >= p->max_jumps) { status = QTO_STATUS_MAXJUMPS; break; }
                double before = norm;
                event_block(s->b->seed, traj_id, (int64_t)n_jumps + 1, wd);
                apply_jump_rule(qto_uniform(wd[0]), qto_uniform(wd[1]), &l, &c);
                /* multiply by the radial part of the collapse operator, r */
                for (int32_t j = 1; j < N; ++j) {
                    double rj = (double)j * dr;
                    w->re[j] *= rj; w->im[j] *= rj;
                }
                double f = 1.0 / sqrt(norm_of(N, dr, w->re, w->im));
                for (int32_t j = 1; j < N; ++j) { w->re[j] *= f; w->im[j] *= f; }
                norm = norm_of(N, dr, w->re, w->im);
                r = qto_uniform(wd[2]);
                n_jumps += 1;
                if (out->jump_log && logged < out->jump_log_cap) {
                    double* e = out->jump_log + ((size_t)i * out->jump_log_cap + logged) * 5;
                    e[0] = (double)n; e[1] = l; e[2] = c; e[3] = before; e[4] = norm;
                    ++logged;
                }
            }
        }
    }

    double ov[6] = { 0, 0, 0, 0, 0, 0 }, sv[6] = { 0, 0, 0, 0, 0, 0 };
    if (status == QTO_STATUS_OK) {
        singlet_overlaps(N, dr, s->basis, l, c, w->re, w->im, ov);
        for (int bb = 0; bb < 6; ++bb)
            /* a state the initial state does not populate (population
               below 1e-12: rounding) has no survival ratio; the overlap
               itself is reported */
            sv[bb] = (s->init_overlap[bb] > 1e-12) ? ov[bb] / s->init_overlap[bb] : ov[bb];
    }
    if (out->norm) out->norm[i] = norm;
    if (out->first_r) out->first_r[i] = first_r;
    if (out->overlap) for (int bb = 0; bb < 6; ++bb) out->overlap[6 * i + bb] = ov[bb];
    if (out->survival) for (int bb = 0; bb < 6; ++bb) out->survival[6 * i + bb] = sv[bb];
    if (out->mean_r) out->mean_r[i] = mean_radius(N, dr, w->re, w->im);
    if (out->l) out->l[i] = l;
    if (out->color) out->color[i] = c;
    if (out->n_jumps) out->n_jumps[i] = n_jumps;
    if (out->status) out->status[i] = status;
    if (out->steps_done) out->steps_done[i] = steps;
    if (out->min_gap) out->min_gap[i] = min_gap;
    if (out->psi) {
        double* dst = out->psi + (size_t)i * 2 * N;
        for (int32_t j = 0; j < N; ++j) { dst[2 * j] = w->re[j]; dst[2 * j + 1] = w->im[j]; }
    }
}

static int validate(const qto_physics* p, const qto_ttable* tt, const qto_init* ini, const qto_batch* b)
{
    if (!p || !tt || !ini || !b) return -1;
    if (p->N < 4 || (p->N & (p->N - 1)) != 0) return -2;
    if (!(p->L > 0) || !(p->dt > 0) || !(p->mass > 0) || !(p->alpha_s >= 0)) return -3;
    if (!(p->kappa_hat >= 0 || p->kappa_hat == -1.0 || p->kappa_hat == -2.0 || p->kappa_hat == -3.0)
        || p->gamma_hat > 0) return -4;
    if (p->deriv_type != 0 && p->deriv_type != 1) return -5;
    if (p->potential != QTO_POTENTIAL_MUNICH && p->potential != QTO_POTENTIAL_KSU) return -5;
    /* the KSU potential is a singlet potential without jumps */
    if (p->potential == QTO_POTENTIAL_KSU &&
        (p->do_jumps || ini->color != QTO_SINGLET || !(p->md_factor > 0))) return -5;
    if (!(p->r_max > 0) || p->r_max > 1) return -6;
    if (!tt->tau || !tt->T || tt->n < 2 || tt->max_steps < 0 || tt->vacuum_steps < 0) return -7;
    for (int32_t k = 0; k + 1 < tt->n; ++k) if (!(tt->tau[k + 1] > tt->tau[k])) return -7;
    if (ini->l < 0 || (ini->color != QTO_SINGLET && ini->color != QTO_OCTET)) return -8;
    if (ini->kind == QTO_INIT_ARRAY && !ini->u_re) return -8;
    if (ini->kind == QTO_INIT_GAUSSIAN && !(ini->width > 0)) return -8;
    if (ini->kind == QTO_INIT_COULOMB && !(p->alpha_s > 0)) return -8;
    if (b->n_traj < 0) return -9;
    return 0;
}

int qto_run(const qto_physics* p, const qto_ttable* tt, const qto_init* ini,
            const qto_batch* b, qto_results* out, int n_threads)
{
    int rc = validate(p, tt, ini, b);
    if (rc != 0) return rc;
    int32_t N = p->N;
    double dr = p->L / (double)N;

    shared_setup s;
    memset(&s, 0, sizeof s);
    s.p = p; s.tt = tt; s.ini = ini; s.b = b; s.out = out;
    s.n_steps = qto_num_steps(p, tt);

    double* tab = sine_table(N);
    double* mom_re = (double*)calloc(N, sizeof(double));
    double* mom_im = (double*)calloc(N, sizeof(double));
    for (int32_t k = 1; k < N; ++k) {
        if (p->flags & QTO_FLAG_KINETIC_OFF) { mom_re[k] = 1.0; mom_im[k] = 0.0; continue; }
        double ph = -kinetic_energy(p, k) * p->dt;   /* exp(-i T_kin dt) */
        mom_re[k] = cos(ph);
        mom_im[k] = sin(ph);
    }
    /* the given projection basis (ProjType 1), else the Coulomb states;
       without a Coulomb term there is no Coulomb basis: overlaps are 0 */
    double* basis = (double*)calloc((size_t)6 * N, sizeof(double));
    if (p->basis)
        memcpy(basis, p->basis, sizeof(double) * 6 * (size_t)N);
    else if (p->alpha_s > 0)
        for (int bb = 0; bb < 6; ++bb)
            qto_basis_state(N, p->L, p->mass, p->alpha_s, BASIS_N[bb], BASIS_L[bb], basis + (size_t)bb * N);
    double* init_re = (double*)calloc(N, sizeof(double));
    double* init_im = (double*)calloc(N, sizeof(double));
    if (initial_state(p, ini, init_re, init_im) != 0) {
        free(tab); free(mom_re); free(mom_im); free(basis); free(init_re); free(init_im);
        return -10;
    }
    /* survival ratios refer to the prepared state, before any vacuum phase */
    singlet_overlaps(N, dr, basis, ini->l, ini->color, init_re, init_im, s.init_overlap);
    s.tab = tab; s.mom_re = mom_re; s.mom_im = mom_im; s.basis = basis;
    s.init_re = init_re; s.init_im = init_im;

    double* buf0 = (double*)calloc((size_t)6 * N, sizeof(double));
    workspace w0;
    w0.re = buf0; w0.im = buf0 + N; w0.tre = buf0 + 2 * N; w0.tim = buf0 + 3 * N;
    w0.fre = buf0 + 4 * N; w0.fim = buf0 + 5 * N;
    /* in-vacuum evolution (T = 0) of the initial state, once, then stored as
       the state every trajectory starts from */
    if (tt->vacuum_steps > 0) {
        memcpy(w0.re, init_re, sizeof(double) * N);
        memcpy(w0.im, init_im, sizeof(double) * N);
        for (int64_t n = 0; n < tt->vacuum_steps; ++n) {
            half_step_factor(p, ini->l, ini->color, 0.0, &w0);
            strang_step(N, tab, &w0, mom_re, mom_im);
        }
        memcpy(init_re, w0.re, sizeof(double) * N);
        memcpy(init_im, w0.im, sizeof(double) * N);
    }
    /* the zeroth trajectory (jumps impossible), its results kept for the
       trajectories that cannot jump */
    qto_results zres;
    memset(&zres, 0, sizeof zres);
    double* zbuf = NULL;
    if (b->no_jump_shortcut && p->do_jumps) {
        int64_t ns = s.n_steps;
        zbuf = (double*)calloc((size_t)(17 + 2 * N + ns), sizeof(double));
        int32_t* zint = (int32_t*)calloc(4, sizeof(int32_t));
        int64_t* zsteps = (int64_t*)calloc(1, sizeof(int64_t));
        zres.norm = zbuf; zres.first_r = zbuf + 1; zres.overlap = zbuf + 2;
        zres.survival = zbuf + 8; zres.mean_r = zbuf + 14; zres.min_gap = zbuf + 15;
        zres.psi = zbuf + 17; zres.norm_trace = ns > 0 ? zbuf + 17 + 2 * N : NULL;
        zres.l = zint; zres.color = zint + 1; zres.n_jumps = zint + 2; zres.status = zint + 3;
        zres.steps_done = zsteps;
        shared_setup sz = s;
        sz.out = &zres;
        run_one(&sz, 0, &w0, 1);
        s.have_zeroth = 1;
        s.r_min = zres.min_gap[0];
        s.zeroth = &zres;
    }

#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel
    {
        workspace w;
        double* buf = (double*)calloc((size_t)6 * N, sizeof(double));
        w.re = buf; w.im = buf + N; w.tre = buf + 2 * N; w.tim = buf + 3 * N;
        w.fre = buf + 4 * N; w.fim = buf + 5 * N;
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < b->n_traj; ++i) run_one(&s, i, &w, 0);
        free(buf);
    }
    if (zbuf) {
        free(zbuf); free(zres.l); free(zres.steps_done);
    }
    free(buf0);
    free(tab); free(mom_re); free(mom_im); free(basis); free(init_re); free(init_im);
    return 0;
}
