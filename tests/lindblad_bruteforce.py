"""Brute-force density-matrix solution of the quarkonium Lindblad equation on
a tiny radial grid, written for the tests with numpy only.

It solves eq. (Lindblad) of the paper in its block-diagonal form
(eq. rhoso): one (N-1)x(N-1) block rho_{c,l} per colour c in {s, o} and
l = 0..l_max.  Each block obeys

    d rho_cl/dt = -i (H_cl rho_cl - rho_cl H_cl^+)
                  + sum_{c', l' = l -+ 1} R(c'->c) p(l'->l) r rho_{c'l'} r

with H_cl = S diag(p^2/M) S + V_R^c(r) + l(l+1)/(M r^2) - (i/2) Gamma_c(r),
Gamma_s = kappa r^2, Gamma_o = (7/16) kappa r^2 (Sec. "Collapse operators,
partial widths, and color state transitions"), feed rates from the collapse
operators of eq. (collapse):  R(s->o) = kappa,  R(o->s) = kappa/8,
R(o->o) = 5 kappa/16, and p(l'->l'-1) = l'/(2l'+1),
p(l'->l'+1) = (l'+1)/(2l'+1) (eq. Pl+-).  Probability that would flow to
l_max + 1 is dropped, so the trace measures the truncation.  Time stepping is
classical RK4.  The state is a dict {(c, l): matrix}.
"""
import numpy as np


def operators(N, L, M, alpha, kappa, gamma):
    j = np.arange(1, N)
    S = np.sqrt(2.0 / N) * np.sin(np.pi * np.outer(j, j) / N)
    p = np.pi * j / L
    r = j * L / N
    kin = S @ np.diag(p * p / M) @ S
    vr = {0: -alpha / r + 0.5 * gamma * r * r, 1: alpha / (8.0 * r) + (7.0 / 32.0) * gamma * r * r}
    width = {0: kappa * r * r, 1: (7.0 / 16.0) * kappa * r * r}
    return kin, vr, width, r


def solve(N, L, M, alpha, kappa, gamma, l_max, rho0, dt, n_steps):
    kin, vr, width, r = operators(N, L, M, alpha, kappa, gamma)
    keys = [(c, l) for c in (0, 1) for l in range(l_max + 1)]
    Heff = {}
    for c, l in keys:
        H = kin + np.diag(vr[c] + l * (l + 1) / (M * r * r))
        Heff[(c, l)] = H - 0.5j * np.diag(width[c])
    rate = {(0, 1): kappa, (1, 0): kappa / 8.0, (1, 1): 5.0 * kappa / 16.0, (0, 0): 0.0}

    def deriv(rho):
        out = {}
        for (c, l) in keys:
            H = Heff[(c, l)]
            d = -1j * (H @ rho[(c, l)] - rho[(c, l)] @ H.conj().T)
            for cs in (0, 1):
                R = rate[(cs, c)]
                if R == 0.0:
                    continue
                for ls, pr in ((l - 1, (l) / (2.0 * l - 1.0) if l >= 1 else 0.0),
                               (l + 1, (l + 1.0) / (2.0 * l + 3.0))):
                    # source l' = l-1 jumps up with p = l'+1 / (2l'+1) = l/(2l-1);
                    # source l' = l+1 jumps down with p = l'/(2l'+1) = (l+1)/(2l+3)
                    if ls < 0 or ls > l_max or pr == 0.0:
                        continue
                    src = rho[(cs, ls)]
                    d = d + R * pr * (r[:, None] * src * r[None, :])
            out[(c, l)] = d
        return out

    def axpy(a, x, y):
        return {k: y[k] + a * x[k] for k in keys}

    rho = {k: np.zeros((N - 1, N - 1), complex) for k in keys}
    for k, v in rho0.items():
        rho[k] = v.astype(complex)
    for _ in range(n_steps):
        k1 = deriv(rho)
        k2 = deriv(axpy(0.5 * dt, k1, rho))
        k3 = deriv(axpy(0.5 * dt, k2, rho))
        k4 = deriv(axpy(dt, k3, rho))
        rho = {k: rho[k] + dt / 6.0 * (k1[k] + 2 * k2[k] + 2 * k3[k] + k4[k]) for k in keys}
    return rho
