/*
 * qtraj_oracle.h -- interface of the CPU reference ("oracle") for the
 * quantum-trajectory (waiting-time Monte-Carlo wave-function) solver of the
 * QTraj 1.0 paper (Ba Omar et al., arXiv:2107.06147).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, FP64 statement
 * of what the method computes.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  The GPU library never links,
 * includes or calls anything from this directory, and this file shares no
 * declarations with the GPU library's public header.
 *
 * Conventions (all natural units, GeV and GeV^-1):
 *   grid      dr = L/N, r_j = j*dr, j = 1..N-1; u(0) = u(L) = 0.  Arrays of
 *             length N are indexed by j, element 0 is the boundary and is 0.
 *   DST-I     (S u)_k = sqrt(2/N) sum_{j=1}^{N-1} u_j sin(pi j k / N).
 *   momenta   p_k = pi k / L, k = 1..N-1.
 *   norm      dr * sum_j |u_j|^2                      (eq. normcond)
 */
#ifndef QTRAJ_ORACLE_H
#define QTRAJ_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { QTO_SINGLET = 0, QTO_OCTET = 1 };
enum { QTO_INIT_COULOMB = 0, QTO_INIT_GAUSSIAN = 1, QTO_INIT_ARRAY = 2 };
enum { QTO_STATUS_OK = 0, QTO_STATUS_RMAX = 1, QTO_STATUS_MAXJUMPS = 2,
       QTO_STATUS_NOJUMP = 4 };   /* 4: results taken from the no-jump trajectory */
enum { QTO_FLAG_KINETIC_OFF = 1 };   /* test flag: kinetic factor := 1 */
enum { QTO_POTENTIAL_MUNICH = 0, QTO_POTENTIAL_KSU = 1 };

typedef struct {
    int32_t N;            /* grid points (N-1 unknowns)                      */
    double  L;            /* box size, GeV^-1                                 */
    double  dt;           /* time step, GeV^-1                                */
    double  mass;         /* heavy-quark mass M; kinetic energy p^2/M         */
    double  alpha_s;      /* strong coupling; alpha = C_F alpha_s             */
    double  kappa_hat;    /* kappa = kappa_hat T^3; -1/-2/-3: the central,
                             lower, upper fit kappa_hat(T) (qto_kappa_hat)    */
    double  gamma_hat;    /* gamma = gamma_hat T^3                            */
    int32_t deriv_type;   /* 0: p^2/M, 1: 2(1-cos(p dr))/(M dr^2)             */
    int32_t do_jumps;     /* 0: H_eff evolution only                          */
    int32_t max_jumps;    /* < 0: unlimited                                   */
    double  r_max;        /* first threshold above r_max: zero overlaps       */
    int32_t flags;        /* QTO_FLAG_*                                       */
    int32_t potential;    /* QTO_POTENTIAL_*: Munich (appendix "Munich
                             potential") or isotropic KSU (appendix
                             "Isotropic KSU potential"; singlet, no jumps)    */
    double  md_factor;    /* KSU: the Debye-mass factor F_mD                  */
    const double* basis;  /* NULL: the Coulomb states; else 6 x N states to
                             project on (ProjType 1: the vacuum eigenstates,
                             see eigen_basis in __init__.py)                  */
} qto_physics;

typedef struct {
    const double* tau;    /* table times, GeV^-1, strictly increasing         */
    const double* T;      /* temperatures, GeV                                */
    int32_t n;            /* table length (>= 2)                              */
    double  tau_start;    /* t_0 of step 0                                    */
    double  T_final;      /* stop once T(t_n) < T_final                       */
    int64_t max_steps;    /* hard cap on the number of steps                  */
    int64_t vacuum_steps; /* steps of in-vacuum evolution (T = 0, no jumps) of
                             the initial state before tau_start, done once for
                             the batch (Sec. "Summary of QTraj execution",
                             step 3: evolution from t0 until the medium)     */
} qto_ttable;

typedef struct {
    int32_t kind;         /* QTO_INIT_*                                       */
    int32_t n;            /* principal quantum number (Coulomb)              */
    int32_t l;            /* angular momentum                                 */
    int32_t color;        /* QTO_SINGLET / QTO_OCTET                          */
    double  width;        /* Gaussian width, GeV^-1                           */
    const double* u_re;   /* QTO_INIT_ARRAY: N values indexed by j           */
    const double* u_im;
} qto_init;

typedef struct {
    int64_t  n_traj;
    uint64_t seed;
    uint64_t traj_id0;    /* trajectory i of the batch has id               */
    uint64_t traj_id_stride; /* traj_id0 + i * traj_id_stride (0 means 1)    */
    int32_t  no_jump_shortcut; /* 1: the zeroth (no-jump) trajectory is run
                             first; a trajectory whose first threshold lies
                             below its smallest norm cannot jump and takes its
                             results (status QTO_STATUS_NOJUMP)              */
} qto_batch;

/* Every pointer may be NULL (output not wanted), except where noted.        */
typedef struct {
    double*  norm;        /* [n_traj] final norm                              */
    double*  first_r;     /* [n_traj] first threshold                         */
    double*  overlap;     /* [6*n_traj] 1S,2S,1P,3S,2P,1D                      */
    double*  survival;    /* [6*n_traj]                                       */
    double*  mean_r;      /* [n_traj]                                         */
    int32_t* l;           /* [n_traj] final l                                 */
    int32_t* color;       /* [n_traj] final colour                            */
    int32_t* n_jumps;     /* [n_traj]                                         */
    int32_t* status;      /* [n_traj] QTO_STATUS_*                            */
    int64_t* steps_done;  /* [n_traj]                                         */
    double*  min_gap;     /* [n_traj] min over decisions of |norm - r|        */
    double*  psi;         /* [2*N*n_traj] final u, (re,im) interleaved        */
    double*  norm_trace;  /* [n_steps*n_traj] norm after every step           */
    int32_t  jump_log_cap;/* entries per trajectory in jump_log               */
    double*  jump_log;    /* [5*cap*n_traj]: step, l', c', norm before, after */
} qto_results;

/* Number of steps the temperature table allows (max_steps cap included). */
int64_t qto_num_steps(const qto_physics* p, const qto_ttable* tt);

/* Runs n_traj trajectories.  Returns 0 on success, a negative code on a
 * rejected input.  n_threads <= 0 uses the OpenMP default. */
int qto_run(const qto_physics* p, const qto_ttable* tt, const qto_init* ini,
            const qto_batch* b, qto_results* out, int n_threads);

/* Pieces exposed for the pin tests. */
void   qto_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
double qto_uniform(uint64_t word);
void   qto_dst1(int32_t N, const double* in_re, const double* in_im,
                double* out_re, double* out_im);
void   qto_jump_rule(uint64_t seed, uint64_t traj_id, int64_t event,
                     int32_t l, int32_t c, int32_t* l_new, int32_t* c_new);
int    qto_basis_state(int32_t N, double L, double mass, double alpha_s,
                       int32_t n, int32_t l, double* u);
double qto_temperature(const qto_ttable* tt, double t);
double qto_kappa_hat(double kappa_hat, double T);
double qto_ksu_phi(double a);
/* V_R + i V_I of the configured potential at r (l, colour c, temperature
 * T), and the kinetic energy of sine mode k (GeV): the two parts of the
 * Hamiltonian, for the vacuum eigenstates. */
void   qto_potential(const qto_physics* p, double r, int32_t l, int32_t c, double T,
                     double* VR, double* VI);
double qto_kinetic_energy(const qto_physics* p, int32_t k);

#ifdef __cplusplus
}
#endif
#endif
