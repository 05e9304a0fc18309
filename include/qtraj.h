/*
 * qtraj.h -- C ABI of the MI355X quantum-trajectory solver.
 *
 * The library evolves many independent radial wave functions u_l(r) of a
 * heavy quark-antiquark pair with the waiting-time Monte-Carlo wave-function
 * method of QTraj 1.0 (Ba Omar et al., arXiv:2107.06147):
 *   - split-step (Strang) pseudo-spectral steps under the non-Hermitian
 *     effective Hamiltonian of the Munich potential (paper: Sec. "Algorithm
 *     for deterministic evolution between quantum jumps", eq. (uUpdate), and
 *     the appendix "Munich potential");
 *   - after each step the norm (eq. (normcond)) is compared with the
 *     trajectory's random threshold; when it has dropped to the threshold a
 *     quantum jump l -> l +- 1, singlet <-> octet is applied with the
 *     probabilities of eqs. (Pl+-) and (pjump) and the state is multiplied by
 *     r and renormalised (Secs. "The waiting time approach" and "Summary of
 *     QTraj execution").
 *
 * Conventions (natural units: GeV, GeV^-1).
 *   grid     dr = L/N, r_j = j dr, j = 1..N-1, u(0) = u(L) = 0.  A wave
 *            function is N complex values indexed by j; element 0 is 0.
 *   kinetic  p_k = pi k / L; E_k = p_k^2 / M (deriv_type 0) or
 *            2 (1 - cos(p_k dr)) / (M dr^2) (deriv_type 1), M the heavy-quark
 *            mass (reduced mass M/2).
 *   potential alpha = (4/3) alpha_s, kappa = kappa_hat T^3, gamma = gamma_hat T^3
 *            singlet V = -alpha/r + gamma r^2/2  - i kappa r^2/2
 *            octet   V = +alpha/(8r) + 7 gamma r^2/32 - i 7 kappa r^2/32
 *            plus l(l+1)/(M r^2).
 *   time     t_n = tau_start + n dt; step n uses T(t_n), linear in the table.
 *   steps    a trajectory takes n_steps = min(max_steps, first n with
 *            t_n > tau[last] or T(t_n) < T_final) steps.
 *   random   Philox4x64-10, key (seed, 0), counter (event+1, trajectory id,
 *            0, 0); event 0 gives the first threshold (word 2), event e >= 1
 *            (the e-th jump) gives u_l (word 0), u_c (word 1) and the next
 *            threshold (word 2); u = ((w >> 12) + 0.5) 2^-52.
 *   jump     iff norm <= threshold; l -> l-1 iff u_l < l/(2l+1), else l+1;
 *            octet -> singlet iff u_c < 2/7, singlet -> octet always.
 *   results  overlaps with the six states 1S,2S,1P,3S,2P,1D of the
 *            projection basis (phys->basis: the Coulomb states of Bohr
 *            radius 2/(M alpha), or the vacuum eigenstates of
 *            qt_eigen_basis), normalised on the grid, of the final
 *            normalised state, non-zero only for a singlet of matching l;
 *            survival = overlap / initial overlap (raw overlap where the
 *            initial overlap is below 1e-12: a state the initial state
 *            does not populate).
 *
 * Threading: a context may be used from one host thread at a time; distinct
 * contexts are independent.  A server (qt_server_*) is thread-safe.
 * Errors: every call returns a qt_status; no call aborts.  qt_last_error()
 * gives a message for the calling thread's last failure.
 */
#ifndef QTRAJ_H
#define QTRAJ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QT_OK = 0,
    QT_EINVAL = 1,      /* an argument failed validation; nothing was run     */
    QT_ENOMEM = 2,      /* device or host allocation failed / over budget     */
    QT_EDEVICE = 3,     /* a HIP runtime call failed                          */
    QT_EBUSY = 4,       /* resource in use                                    */
    QT_ETIMEOUT = 5,    /* qt_wait ran out of time                            */
    QT_ECANCELED = 6,   /* the request was cancelled                          */
    QT_ENOTFOUND = 7,   /* unknown request id                                 */
    QT_ENOCONV = 8      /* an iterative solver did not converge               */
} qt_status;

typedef enum { QT_FP64 = 0, QT_FP32_BULK = 1 } qt_precision;
/* FUSED: one persistent kernel, state in registers/LDS for the whole run.
 * PLAIN: one kernel per sub-step per time step, state in HBM (FP64 only). */
typedef enum { QT_FORM_FUSED = 0, QT_FORM_PLAIN = 1 } qt_form;
typedef enum { QT_INIT_COULOMB = 0, QT_INIT_GAUSSIAN = 1, QT_INIT_ARRAY = 2, QT_INIT_EIGEN = 3 } qt_init_kind;

/* Projection basis of the overlaps and survival probabilities (paper:
 * ProjType 0 and 1). */
typedef enum { QT_BASIS_COULOMB = 0, QT_BASIS_EIGEN = 1 } qt_basis_kind;
typedef enum { QT_SINGLET = 0, QT_OCTET = 1 } qt_color;
/* LMAX: l exceeded the tabulated range (l > 255; ends like MAXJUMPS).
 * NOJUMP: the first threshold lies below every norm of the batch's no-jump
 * (zeroth) trajectory, so the trajectory cannot jump: its results are that
 * trajectory's (no_jump_shortcut; paper: Sec. "Summary of QTraj execution",
 * step 4, r_0 < rMin = p_NoJumps). */
typedef enum { QT_TRAJ_OK = 0, QT_TRAJ_RMAX = 1, QT_TRAJ_MAXJUMPS = 2, QT_TRAJ_LMAX = 3,
               QT_TRAJ_NOJUMP = 4 } qt_traj_status;
enum { QT_FLAG_KINETIC_OFF = 1 };   /* kinetic factor := 1 (test special case) */
/* MUNICH: appendix "Munich potential" (singlet/octet, jumps).  KSU: appendix
 * "Isotropic KSU potential": screened Karsch-Mehr-Satz real part with string
 * breaking at 1.25 fm (a = 0.409, sigma = 0.21 GeV^2), imaginary part
 * -alpha_s C_F T phi(m_D r); alpha_s(2 pi T) at one loop from
 * alpha_s(5 GeV) = 0.2034 with 3 light flavours; Debye mass
 * m_D = md_factor T sqrt(N_c (1 + N_F/6) pi (4/3) alpha_s).  Singlet only,
 * no jumps (do_jumps = 0); no medium where T = 0 or below the coupling's
 * one-loop pole. */
typedef enum { QT_POTENTIAL_MUNICH = 0, QT_POTENTIAL_KSU = 1 } qt_potential;

/* Physics and grid (paper: table "Code parameters", groups Physics, Jump,
 * Grid).  Valid: N a power of two in [256, 8192]; L, dt, mass > 0;
 * alpha_s >= 0; kappa_hat >= 0, or -1, -2, -3 for the central, lower and
 * upper fit kappa_hat(T) = 1/(a x^{3/2} + b x + c x^{1/2} + d), x = T/T_c,
 * T_c = 155 MeV (appendix "Munich potential"; 0 where the denominator is
 * not positive); gamma_hat <= 0; deriv_type 0 or 1; 0 < r_max <= 1;
 * max_jumps < 0 means unlimited. */
typedef struct {
    int32_t N;
    double  L, dt, mass, alpha_s, kappa_hat, gamma_hat;
    int32_t deriv_type, do_jumps, max_jumps;
    double  r_max;
    int32_t flags;
    int32_t potential;     /* qt_potential */
    double  md_factor;     /* KSU: > 0 */
    int32_t basis;         /* qt_basis_kind: the states the overlaps project on,
                              the analytic Coulomb states or the vacuum
                              eigenstates of qt_eigen_basis (computed on the
                              device at the first use, cached per context) */
    int32_t pad0;
} qt_physics;

/* Temperature table (paper: Temperature parameters).  Host pointers, read
 * during the call.  tau in GeV^-1 strictly increasing, n >= 2.
 * vacuum_steps >= 0: before tau_start the initial state is evolved that many
 * steps in vacuum (T = 0, no jumps), once for the batch, and every
 * trajectory starts from the result (paper: Sec. "Summary of QTraj
 * execution", step 3, evolution from t0 until the medium turns on; the
 * count is (t_med - t0)/dt).  Survival ratios still refer to the prepared
 * initial state. */
typedef struct {
    const double* tau;
    const double* T;
    int32_t n;
    double  tau_start, T_final;
    int64_t max_steps;
    int64_t vacuum_steps;
} qt_ttable;

/* Initial state (paper: Initial condition parameters).  COULOMB: hydrogen-
 * like (n, l) for n <= 3; GAUSSIAN: r^{l+1} exp(-r^2/(2 width^2)); ARRAY:
 * u_re/u_im host arrays of N values indexed by j (u_im may be NULL); EIGEN
 * (paper: initType 100): the vacuum eigenstate (n, l) of qt_eigen_basis,
 * one of 1S, 2S, 1P (n=2), 3S, 2P (n=3), 1D (n=3), singlet.  Every initial
 * state is normalised on the grid. */
typedef struct {
    int32_t kind, n, l, color;
    double  width;
    const double* u_re;
    const double* u_im;
} qt_init;

/* Trajectory i of a batch has id traj_id0 + i * traj_id_stride (stride 0 is
 * read as 1); ids select the random streams, so results do not depend on
 * how trajectories are batched.  precision: qt_precision; form: qt_form.
 * no_jump_shortcut = 1 (qt_run / qt_run_many, FUSED form, jumps on): the
 * batch's zeroth trajectory (the same evolution with no jumps) runs first;
 * a trajectory whose first threshold lies below its smallest norm takes its
 * results, status QT_TRAJ_NOJUMP, exactly as if it had been evolved. */
typedef struct {
    int64_t  n_traj;
    uint64_t seed, traj_id0, traj_id_stride;
    int32_t  precision, form;
    int32_t  no_jump_shortcut;
} qt_batch;

/* Per-trajectory outputs, DEVICE pointers owned by the caller.  Any pointer
 * may be NULL.  overlap/survival hold 6 values per trajectory; psi holds N
 * complex doubles (re, im interleaved) per trajectory; min_gap is the
 * smallest |norm - threshold| over all jump decisions (diagnostic for
 * comparisons near the threshold).
 * jump_log (qt_run and qt_run_many only; NULL for jobs and the server) holds
 * jump_log_cap entries of 3 int32 per trajectory, entry e of trajectory i at
 * jump_log[3 (i jump_log_cap + e)]: the step n (0-based) after which the
 * e-th jump happened, and l and colour after it (paper: Sec. "The waiting
 * time approach": the jump times of the waiting-time method; Sec. "Summary
 * of QTraj execution", step 4).  The first min(n_jumps, jump_log_cap)
 * entries are written, the rest are left as they were.  jump_log_cap >= 0. */
typedef struct {
    double  *norm, *first_r, *overlap, *survival, *mean_r;
    int32_t *l, *color, *n_jumps, *status;
    int64_t *steps_done;
    double  *min_gap;
    double  *psi;
    int32_t *jump_log;
    int32_t  jump_log_cap;
    int32_t  pad0;
} qt_results;

typedef struct qt_context qt_context;
typedef struct qt_job qt_job;
typedef struct qt_server qt_server;

/* Creates a context on HIP device `device` (ordinal).  QT_EDEVICE if the
 * device does not exist. */
qt_status qt_context_create(int device, qt_context** out);
qt_status qt_context_destroy(qt_context* ctx);

/* Runs one batch to completion, stream-ordered on `hip_stream` (a
 * hipStream_t; NULL = default stream): validates, builds the tables on the
 * host, uploads them and launches the kernels.  Results are valid once the
 * stream reaches this point.  Host inputs may be freed when the call
 * returns. */
qt_status qt_run(qt_context* ctx, const qt_physics* phys, const qt_ttable* tt,
                 const qt_init* init, const qt_batch* batch, const qt_results* dev_out,
                 void* hip_stream);

/* Several batches of possibly different N and lifetimes in one job: every
 * batch keeps its own physics, table and initial state; trajectories are
 * scheduled longest-first on persistent workgroups that refill from a
 * device queue.  All batches must have the same precision, FUSED form. */
qt_status qt_run_many(qt_context* ctx, int32_t n_batches, const qt_physics* phys,
                      const qt_ttable* tt, const qt_init* init, const qt_batch* batch,
                      const qt_results* dev_out, void* hip_stream);

/* Segmented runs with checkpoints (FUSED form).  A job holds every
 * trajectory's state (wave function, step, l, colour, threshold, counters)
 * in device memory between segments.  qt_job_advance runs every unfinished
 * trajectory for `steps` more steps, or to its end if that comes first (a
 * replay of a captured HIP graph of launches of `segment_steps` steps each,
 * the last one of the remainder when `steps` is not a multiple), then the
 * state is a
 * checkpoint: qt_job_save copies it to `dst` (host or device, state_bytes),
 * qt_job_load restores it into a job created with identical arguments. */
qt_status qt_job_create(qt_context* ctx, const qt_physics* phys, const qt_ttable* tt,
                        const qt_init* init, const qt_batch* batch, int64_t segment_steps,
                        qt_job** out);
qt_status qt_job_advance(qt_job* job, int64_t steps, void* hip_stream);
qt_status qt_job_done(qt_job* job, int32_t* done);             /* synchronises */
qt_status qt_job_state_bytes(qt_job* job, size_t* bytes);
qt_status qt_job_save(qt_job* job, void* dst, void* hip_stream);
qt_status qt_job_load(qt_job* job, const void* src, void* hip_stream);
qt_status qt_job_results(qt_job* job, const qt_results* dev_out, void* hip_stream);
qt_status qt_job_destroy(qt_job* job);

/* Continuous-batching server.  Requests (a batch each) are admitted while
 * others run, in arrival order, as device memory within hbm_budget_bytes and
 * persistent slots free up: a request is admitted while the admitted
 * trajectories, counted against the device's resident slots of their grid
 * size (compute units times workgroups per CU of the kernel variant), stay
 * within max_occupancy; when nothing runs, the next request is admitted
 * whatever its size.  Admission happens at segment boundaries of
 * segment_steps steps.
 * qt_submit copies its inputs and returns at once; qt_wait copies a finished
 * request's results to HOST pointers.  A request that could not run (its
 * device memory could not be allocated at admission, a launch or the copy
 * of its results failed) ends with that cause: qt_wait returns QT_ENOMEM or
 * QT_EDEVICE for it, QT_ECANCELED only after qt_cancel.  The kernel variant
 * of each grid size is fixed at its first use for the server's life. */
typedef struct {
    size_t  hbm_budget_bytes;     /* 0: 50% of free device memory             */
    int64_t segment_steps;        /* steps per admission round (e.g. 500)     */
    int32_t precision;            /* qt_precision of every request            */
    int32_t pad0;
    double  max_occupancy;        /* admitted trajectories per resident slot; 0:
                                     8 (< 0: no slot limit, memory only).  A
                                     round runs every admitted trajectory
                                     segment_steps steps, a whole number of
                                     them per slot: at k per slot the device
                                     is about k / ceil(k) busy            */
} qt_server_cfg;

typedef struct {
    double   p50_latency_s, p99_latency_s, mean_latency_s;
    double   traj_steps_per_s;    /* completed trajectory-steps / busy time   */
    int64_t  completed, admitted, queued, running;
    int64_t  traj_steps;
    size_t   hbm_in_use;
} qt_stats;

qt_status qt_server_create(qt_context* ctx, const qt_server_cfg* cfg, qt_server** out);
qt_status qt_submit(qt_server* s, const qt_physics* phys, const qt_ttable* tt,
                    const qt_init* init, const qt_batch* batch, uint64_t* request_id);
qt_status qt_poll(qt_server* s, uint64_t id, int32_t* done);
qt_status qt_wait(qt_server* s, uint64_t id, const qt_results* host_out, double timeout_s);
qt_status qt_cancel(qt_server* s, uint64_t id);
qt_status qt_server_stats(qt_server* s, qt_stats* out);
qt_status qt_server_destroy(qt_server* s);

/* Number of time steps a run takes with this temperature table (paper: Sec.
 * "Summary of QTraj execution": the evolution runs from tau_start in steps
 * of dt while t_n = tau_start + n dt lies within the table and T(t_n), linear
 * between the table's points, is at least T_final; at most max_steps).
 * Uses phys->dt only.  Host computation, no device work, no context.
 * QT_EINVAL for a null argument, dt not finite and > 0, or an invalid table
 * (as qt_run). */
qt_status qt_count_steps(const qt_physics* phys, const qt_ttable* ttable, int64_t* n_steps);

/* Kernel timing of the most recent qt_run / qt_job_advance on this context:
 * milliseconds between HIP events recorded around its kernel launches on
 * the caller's stream (synchronises that stream). */
qt_status qt_last_kernel_ms(qt_context* ctx, double* ms, int64_t* launches);

/* Kernel variant chosen for (N, precision): threads per trajectory and
 * resident trajectories per CU.  tune=1 measures the candidates first
 * (runs kernels on the context's device). */
qt_status qt_plan(qt_context* ctx, int32_t N, int32_t precision, int32_t tune,
                  int32_t* threads_per_traj, int32_t* traj_per_cu);

/* Kernel variants of the fused form (Munich potential) for (N, precision):
 * threads per trajectory of each, ascending, the first min(cap, count)
 * written to threads (caller-owned, may be null when cap is 0); *count gets
 * how many there are (0 for an N or precision without fused kernels).  Host
 * query: no device work, no context.  The KSU potential has one variant per
 * N, chosen by the library.  QT_EINVAL for a null count or a negative cap. */
qt_status qt_plan_variants(int32_t N, int32_t precision, int32_t* threads, int32_t cap,
                           int32_t* count);

/* Fixes the kernel variant that runs (N, precision) on this context: one of
 * the threads-per-trajectory values of qt_plan_variants, instead of the
 * default or the tuned one (a later qt_plan with tune=1 keeps it).  For
 * reproducible launch configurations, and to test every variant.  Queries
 * the device's residency of that kernel.  QT_EINVAL for a null context or
 * a variant that does not exist; QT_EDEVICE if the kernel cannot be
 * resident. */
qt_status qt_plan_set(qt_context* ctx, int32_t N, int32_t precision, int32_t threads_per_traj);

/* Vacuum eigenstates 1S, 2S, 1P, 3S, 2P, 1D of the discrete Hamiltonian
 * (paper: Sec. "Using the built-in eigensolvers"; the states that initType
 * 100 starts from and ProjType 1 projects on).  The Hamiltonian is the one
 * the evolution integrates at T = 0 for a singlet: the kinetic energy of
 * phys->deriv_type, diagonal in the sine modes of the grid r_m = m dr
 * (dr = L/N, m = 1..N-1, u_0 = u_N = 0), plus the vacuum potential of
 * phys->potential (Munich: -(4/3) alpha_s / r; KSU: the Cornell potential
 * with string breaking) and l(l+1)/(M r^2).  Uses phys->N (256, 512, ...,
 * 8192), L, mass, alpha_s, deriv_type and potential; the rest is ignored.
 * Output (host memory, caller-owned): energies[6] in GeV (binding energies:
 * the state's mass is 2 M + energy) and basis[6 * N], row s the state s as
 * u_m, m = 0..N-1, normalised to dr sum u_m^2 = 1 with u_1 > 0.  Runs
 * kernels on the context's device and returns when done.  QT_EINVAL for an
 * unsupported N or non-positive L or mass; QT_ENOCONV if the iteration
 * does not converge. */
qt_status qt_eigen_basis(qt_context* ctx, const qt_physics* phys, double* energies,
                         double* basis);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): qt_run of
 * the FUSED form without any device allocation.  Its per-call device data
 * (queue counter, work items, the batch's descriptor and tables) goes into
 * one static device buffer of QT_NOALLOC_BUFFER_BYTES that each device
 * holds for the life of the process.  Every call on a device shares that
 * buffer, so calls that overlap on one device race: issue them on one
 * stream, or otherwise one after another.  The context's cached device
 * tables of the grid must exist already, built by an earlier qt_run (or
 * qt_eigen_basis) on the same context with the same N, precision, L, mass,
 * alpha_s, dt and potential: a call that would have to build one returns
 * QT_EINVAL instead.  Also QT_EINVAL: the PLAIN form, no_jump_shortcut,
 * vacuum_steps > 0, or a batch whose items and tables exceed the buffer
 * (12 bytes per trajectory plus about 48 N + 16 n_tab bytes of tables:
 * about 1.3 million trajectories at N = 2048).  Results, status and timing
 * as qt_run; stream-ordered on hip_stream (the staging copy of the host
 * tables synchronises it). */
#define QT_NOALLOC_BUFFER_BYTES (16u << 20)
qt_status qt_run_noalloc(qt_context* ctx, const qt_physics* phys, const qt_ttable* tt,
                         const qt_init* init, const qt_batch* batch, const qt_results* dev_out,
                         void* hip_stream);

const char* qt_last_error(void);
const char* qt_version(void);

#ifdef __cplusplus
}
#endif
#endif
