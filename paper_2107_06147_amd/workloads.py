"""Seeded synthetic inputs for the quantum-trajectory solver.

This module only generates inputs: physics parameters, temperature tables
T(tau), trajectory counts, seeds and request streams.  It holds none of the
solver's arithmetic, so both the GPU library and the CPU oracle can be fed
from it without sharing any of the method's code.

Units are natural (GeV, GeV^-1).  Times quoted in fm/c are converted with
hbar c = 0.1973269804 GeV fm.  The hydrodynamic temperature files of the
paper's examples are not available, so Bjorken profiles T0 (tau0/tau)^(1/3)
(the paper's benchmark medium) and seeded random-walk profiles stand in for
them.

Every config is a plain dict with the keys
  N, L, dt, mass, alpha_s, kappa_hat, gamma_hat, deriv_type, do_jumps,
  max_jumps, r_max, flags, potential, md_factor,
  tau, T, tau_start, T_final, max_steps, vacuum_steps,
  init_kind, init_n, init_l, init_color, init_width,
  n_traj, seed, traj_id0, traj_id_stride, no_jump_shortcut
"""
from __future__ import annotations

import numpy as np

HBARC = 0.1973269804          # GeV fm
FM = 1.0 / HBARC              # 1 fm/c in GeV^-1
MASS_B = 4.65                 # bottom-quark mass, GeV
ALPHA_S = 0.3

SINGLET, OCTET = 0, 1
POTENTIAL_MUNICH, POTENTIAL_KSU = 0, 1
INIT_COULOMB, INIT_GAUSSIAN, INIT_ARRAY, INIT_EIGEN = 0, 1, 2, 3
BASIS_COULOMB, BASIS_EIGEN = 0, 1


def base(**kw):
    cfg = dict(N=512, L=40.0, dt=0.001, mass=MASS_B, alpha_s=ALPHA_S, kappa_hat=4.0,
               gamma_hat=0.0, deriv_type=0, do_jumps=1, max_jumps=-1, r_max=1.0, flags=0,
               potential=0, md_factor=1.0, basis=0,
               tau=np.array([0.0, 1.0e9]), T=np.array([0.4, 0.4]), tau_start=0.0,
               T_final=0.0, max_steps=1000, vacuum_steps=0,
               init_kind=INIT_COULOMB, init_n=1, init_l=0, init_color=SINGLET, init_width=0.0,
               n_traj=16, seed=1, traj_id0=0, traj_id_stride=1, no_jump_shortcut=0)
    cfg.update(kw)
    return cfg


def constant_T(T, n_steps):
    """Table for a constant temperature run of exactly n_steps steps."""
    return dict(tau=np.array([0.0, 1.0e9]), T=np.array([float(T), float(T)]),
                tau_start=0.0, T_final=0.0, max_steps=int(n_steps))


def bjorken_table(T0, tau0_fm, Tf, n_points=500):
    """Bjorken cooling T0 (tau0/tau)^(1/3) sampled uniformly in tau from tau0
    to the time where T reaches Tf.  Returns (tau [GeV^-1], T [GeV])."""
    tau_end_fm = tau0_fm * (T0 / Tf) ** 3
    tau_fm = np.linspace(tau0_fm, tau_end_fm, n_points)
    T = T0 * (tau0_fm / tau_fm) ** (1.0 / 3.0)
    return tau_fm * FM, T


def random_walk_table(rng, n_points=200, tau0_fm=0.6, tau1_fm=2.6, lo=0.2, hi=0.6):
    """Seeded smoothed random walk: T0 ~ U[0.3, 0.5], Gaussian increments of
    0.02 GeV reflected into [lo, hi], then a 5-point moving average."""
    T = np.empty(n_points)
    T[0] = rng.uniform(0.3, 0.5)
    for i in range(1, n_points):
        x = T[i - 1] + rng.normal(0.0, 0.02)
        while x < lo or x > hi:
            x = 2 * lo - x if x < lo else 2 * hi - x
        T[i] = x
    pad = np.concatenate([[T[0]] * 2, T, [T[-1]] * 2])
    T = np.convolve(pad, np.ones(5) / 5.0, mode="valid")
    tau = np.linspace(tau0_fm, tau1_fm, n_points) * FM
    return tau, T


# --------------------------------------------------------------------------
# The workloads.
# --------------------------------------------------------------------------

def c1_parity():
    """16 trajectories, N=512, L=40, dt=0.001, 1000 steps, T=0.4 constant,
    kappa_hat=4, gamma_hat=0, Coulomb 1S singlet, jumps, seed 1."""
    return base(N=512, L=40.0, dt=0.001, kappa_hat=4.0, gamma_hat=0.0,
                init_kind=INIT_COULOMB, init_n=1, init_l=0, init_color=SINGLET,
                n_traj=16, seed=1, **constant_T(0.4, 1000))


def c2_headline(kappa_hat=4.0, gamma_hat=0.0, n_traj=4096, seed=1):
    """4096 trajectories, N=2048, L=40, dt=0.001, Bjorken 0.425 GeV at
    0.6 fm/c down to 0.25 GeV (500 table points, 11,899 steps), Gaussian
    l=0 singlet of width 0.2 fm."""
    tau, T = bjorken_table(0.425, 0.6, 0.25, 500)
    return base(N=2048, L=40.0, dt=0.001, kappa_hat=kappa_hat, gamma_hat=gamma_hat,
                tau=tau, T=T, tau_start=float(tau[0]), T_final=0.25, max_steps=2**62,
                init_kind=INIT_GAUSSIAN, init_l=0, init_color=SINGLET, init_width=0.2 * FM,
                n_traj=n_traj, seed=seed)


C2_RUNS = [(1.0, 0.0), (1.0, -2.0), (4.0, 0.0), (4.0, -2.0)]


def c3_uneven(n_traj=16384, seed=2):
    """Uneven batch: per trajectory N in {1024, 2048, 4096} (L = 20/40/80, so
    dr = 5/256 fixed), l in {0, 1}, T0 ~ U[0.3, 0.55] GeV and
    tau0 ~ U[0.4, 0.8] fm/c (Bjorken down to 0.25 GeV, 500 points).
    Returns a list of single-trajectory configs with trajectory ids 0..n-1."""
    rng = np.random.default_rng(seed)
    Ns = rng.choice([1024, 2048, 4096], size=n_traj)
    ls = rng.integers(0, 2, size=n_traj)
    T0s = rng.uniform(0.3, 0.55, size=n_traj)
    tau0s = rng.uniform(0.4, 0.8, size=n_traj)
    out = []
    for i in range(n_traj):
        N = int(Ns[i])
        tau, T = bjorken_table(float(T0s[i]), float(tau0s[i]), 0.25, 500)
        out.append(base(N=N, L=N * 5.0 / 256.0, dt=0.001, kappa_hat=4.0, gamma_hat=0.0,
                        tau=tau, T=T, tau_start=float(tau[0]), T_final=0.25,
                        max_steps=2**62, init_kind=INIT_GAUSSIAN, init_l=int(ls[i]),
                        init_color=SINGLET, init_width=0.2 * FM, n_traj=1, seed=seed,
                        traj_id0=i))
    return out


def c4_requests(duration_s=120.0, rate=20.0, arrival_seed=4):
    """Served stream: Poisson arrivals; each request holds
    K = clip(round(512 e^Z), 64, 4096) trajectories, N in {1024, 2048}
    (L = 20/40), Gaussian l=0 singlet, its own 200-point random-walk T table
    over tau in [0.6, 2.6] fm/c; request seed 1000 + index.
    Returns a list of (arrival_time_s, config)."""
    rng = np.random.default_rng(arrival_seed)
    t = 0.0
    reqs = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration_s:
            break
        idx = len(reqs)
        rr = np.random.default_rng(1000 + idx)
        K = int(np.clip(round(512.0 * np.exp(rr.normal())), 64, 4096))
        N = int(rr.choice([1024, 2048]))
        tau, T = random_walk_table(rr)
        cfg = base(N=N, L=N * 5.0 / 256.0, dt=0.001, kappa_hat=4.0, gamma_hat=0.0,
                   tau=tau, T=T, tau_start=float(tau[0]), T_final=0.0, max_steps=2**62,
                   init_kind=INIT_GAUSSIAN, init_l=0, init_color=SINGLET,
                   init_width=0.2 * FM, n_traj=K, seed=1000 + idx)
        reqs.append((t, cfg))
    return reqs


def c5_roofline(n_traj=65536, n_steps=20000):
    """65536 trajectories, N=4096, L=60, dt=0.0005, T=0.5 constant,
    kappa_hat=4, gamma_hat=0; initial states cycle 1S/2S/1P singlet
    (trajectory i gets state i mod 3).  Returns three configs, one per
    initial state, with trajectory ids b, b+3, b+6, ..."""
    out = []
    for b, (n, l) in enumerate([(1, 0), (2, 0), (2, 1)]):
        k = len(range(b, n_traj, 3))
        out.append(base(N=4096, L=60.0, dt=0.0005, kappa_hat=4.0, gamma_hat=0.0,
                        init_kind=INIT_COULOMB, init_n=n, init_l=l, init_color=SINGLET,
                        n_traj=k, seed=5, traj_id0=b, traj_id_stride=3,
                        **constant_T(0.5, n_steps)))
    return out
