/* Drives the CPU oracle through its code paths under the address and
 * undefined-behaviour sanitizers (built by tests/test_oracle_sanitizers.py
 * with gcc -fsanitize=address,undefined).  Each case runs a small batch with
 * every output array present; the program prints one line per case and
 * exits non-zero if a run is rejected.  Any sanitizer report aborts it. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "qtraj_oracle.h"

typedef struct {
    const char* name;
    qto_physics p;
    qto_ttable t;
    qto_init i;
    qto_batch b;
} Case;

static int run_case(const Case* c)
{
    const int64_t n = c->b.n_traj;
    const int32_t N = c->p.N;
    const int64_t steps = qto_num_steps(&c->p, &c->t);
    const int32_t cap = 4;
    qto_results r;
    memset(&r, 0, sizeof r);
    r.norm = calloc(n, sizeof(double));
    r.first_r = calloc(n, sizeof(double));
    r.overlap = calloc(6 * n, sizeof(double));
    r.survival = calloc(6 * n, sizeof(double));
    r.mean_r = calloc(n, sizeof(double));
    r.l = calloc(n, sizeof(int32_t));
    r.color = calloc(n, sizeof(int32_t));
    r.n_jumps = calloc(n, sizeof(int32_t));
    r.status = calloc(n, sizeof(int32_t));
    r.steps_done = calloc(n, sizeof(int64_t));
    r.min_gap = calloc(n, sizeof(double));
    r.psi = calloc(2 * (size_t)N * n, sizeof(double));
    r.norm_trace = calloc((size_t)(steps > 0 ? steps : 1) * n, sizeof(double));
    r.jump_log_cap = cap;
    r.jump_log = calloc(5 * (size_t)cap * n, sizeof(double));
    const int rc = qto_run(&c->p, &c->t, &c->i, &c->b, &r, 2);
    double sum = 0.0;
    int jumps = 0;
    for (int64_t k = 0; k < n; ++k) {
        sum += r.norm[k] + r.mean_r[k];
        jumps += r.n_jumps[k];
    }
    printf("%-12s rc=%d steps=%lld jumps=%d checksum=%.12f\n", c->name, rc, (long long)steps,
           jumps, sum);
    free(r.norm); free(r.first_r); free(r.overlap); free(r.survival); free(r.mean_r);
    free(r.l); free(r.color); free(r.n_jumps); free(r.status); free(r.steps_done);
    free(r.min_gap); free(r.psi); free(r.norm_trace); free(r.jump_log);
    return rc;
}

int main(void)
{
    static const double tau_c[2] = {0.0, 1.0e9}, T_c[2] = {0.5, 0.5};
    static double tau_b[40], T_b[40];
    for (int k = 0; k < 40; ++k) {
        tau_b[k] = 3.0 + 0.05 * k;
        T_b[k] = 0.45 * pow(3.0 / tau_b[k], 1.0 / 3.0);
    }
    static double u_re[128], u_im[128];
    for (int j = 0; j < 128; ++j) {
        u_re[j] = sin(3.14159265358979 * 3 * j / 128.0);
        u_im[j] = 0.1 * sin(3.14159265358979 * 5 * j / 128.0);
    }
    const qto_physics base = {128, 12.0, 0.002, 4.65, 0.3, 20.0, 0.0, 0, 1, -1, 1.0, 0,
                              QTO_POTENTIAL_MUNICH, 1.0, NULL};
    const qto_ttable tc = {tau_c, T_c, 2, 0.0, 0.0, 150, 0};
    const qto_ttable tb = {tau_b, T_b, 40, 3.0, 0.3, 100000, 0};
    const qto_init coul = {QTO_INIT_COULOMB, 1, 0, QTO_SINGLET, 0.0, NULL, NULL};
    const qto_init gauss_o = {QTO_INIT_GAUSSIAN, 1, 2, QTO_OCTET, 1.0, NULL, NULL};
    const qto_init arr = {QTO_INIT_ARRAY, 1, 1, QTO_SINGLET, 0.0, u_re, u_im};
    const qto_batch b = {5, 7, 0, 1, 0};
    Case cases[10];
    int nc = 0;
    cases[nc++] = (Case){"jumps", base, tc, coul, b};
    cases[nc] = (Case){"bjorken", base, tb, gauss_o, b};
    cases[nc].p.gamma_hat = -2.0; cases[nc].p.deriv_type = 1; ++nc;
    cases[nc] = (Case){"kappa_fit", base, tb, arr, b};
    cases[nc].p.kappa_hat = -3.0; ++nc;
    cases[nc] = (Case){"maxjumps", base, tc, coul, b};
    cases[nc].p.max_jumps = 1; cases[nc].b.traj_id_stride = 3; ++nc;
    cases[nc] = (Case){"rmax", base, tc, coul, b};
    cases[nc].p.r_max = 0.3; ++nc;
    cases[nc] = (Case){"shortcut", base, tc, coul, b};
    cases[nc].b.no_jump_shortcut = 1; cases[nc].b.n_traj = 9; ++nc;
    cases[nc] = (Case){"vacuum", base, tc, gauss_o, b};
    cases[nc].t.vacuum_steps = 30; ++nc;
    cases[nc] = (Case){"kinetic_off", base, tc, coul, b};
    cases[nc].p.flags = QTO_FLAG_KINETIC_OFF; ++nc;
    cases[nc] = (Case){"ksu", base, tb, coul, b};
    cases[nc].p.potential = QTO_POTENTIAL_KSU; cases[nc].p.do_jumps = 0;
    cases[nc].p.md_factor = 1.2; ++nc;
    cases[nc] = (Case){"empty", base, tc, coul, b};
    cases[nc].b.n_traj = 1; cases[nc].t.max_steps = 0; ++nc;
    int bad = 0;
    for (int k = 0; k < nc; ++k) bad |= run_case(&cases[k]) != 0;
    double d[2 * 16];
    double x[16], y[16];
    for (int j = 0; j < 16; ++j) { x[j] = j; y[j] = -j; }
    qto_dst1(16, x, y, d, d + 16);
    printf("dst %.6f\n", d[3]);
    return bad;
}
