"""GPU parity: the HIP library (through the C ABI) against the CPU oracle,
element by element on the same seeded inputs.  Marked `gpu`."""
import numpy as np
import pytest

import oracle
from paper_2107_06147_amd import qtraj as qt
from paper_2107_06147_amd import workloads as W
from tests.gpu_parity import FP32_DELTA, FP64_DELTA, compare, gpu_run

pytestmark = pytest.mark.gpu

F64, F32 = qt.QT_FP64, qt.QT_FP32_BULK
FUSED, PLAIN = qt.QT_FORM_FUSED, qt.QT_FORM_PLAIN


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = qt.Context(0)
    yield c
    c.close()


JLOG = 64      # jump-log entries per trajectory in the parity runs


@pytest.fixture(scope="module")
def c1_ref():
    return oracle.run(W.c1_parity(), want_psi=True, jump_log_cap=JLOG)


# ---------------------------------------------------- C1: the parity config

@pytest.mark.parametrize("prec,form", [(F64, FUSED), (F64, PLAIN), (F32, FUSED)])
def test_c1_all_trajectories(ctx, c1_ref, prec, form):
    """16 trajectories, N=512, 1000 steps, Coulomb 1S, kappa_hat=4: every
    trajectory, every output."""
    out = gpu_run(ctx, W.c1_parity(), prec, form, jump_log_cap=JLOG)
    st = compare(c1_ref, out, prec, label="c1 prec=%d form=%d" % (prec, form))
    print("c1", prec, form, st)
    assert c1_ref["n_jumps"].sum() > 0          # the case exercises jumps
    assert st["jumps_logged"] > 0               # jump sequences compared
    assert st["near"] <= st["n"] // 2


# ---------------------------------------------------- edge and special cases

def _edge_cases():
    bj_tau, bj_T = W.bjorken_table(0.425, 0.6, 0.25, 500)
    bj = dict(tau=bj_tau, T=bj_T, tau_start=float(bj_tau[0]), T_final=0.25, max_steps=300)
    small = dict(N=256, L=20.0, dt=0.001, kappa_hat=20.0, seed=9)
    return {
        "ragged_3": W.base(n_traj=3, **small, **W.constant_T(0.5, 300)),
        "octet_gauss_l2": W.base(n_traj=6, init_kind=W.INIT_GAUSSIAN, init_l=2, init_color=W.OCTET,
                                 init_width=1.0, **small, **W.constant_T(0.5, 300)),
        "deriv1_gamma_bjorken": W.base(n_traj=6, deriv_type=1, gamma_hat=-2.0,
                                       **dict(small, kappa_hat=4.0), **bj),
        "kinetic_off": W.base(n_traj=4, flags=qt.QT_FLAG_KINETIC_OFF, **small,
                              **W.constant_T(0.5, 200)),
        "rmax": W.base(n_traj=12, r_max=0.4, **small, **W.constant_T(0.5, 200)),
        "maxjumps_1": W.base(n_traj=12, max_jumps=1, **small, **W.constant_T(0.5, 400)),
        "no_jumps": W.base(n_traj=2, do_jumps=0, **small, **W.constant_T(0.5, 300)),
        "zero_steps": W.base(n_traj=5, **small, **W.constant_T(0.5, 0)),
        "stride_ids": W.base(n_traj=7, traj_id0=5, traj_id_stride=3, **small,
                             **W.constant_T(0.5, 200)),
        "coulomb_2p": W.base(n_traj=5, init_kind=W.INIT_COULOMB, init_n=3, init_l=1, **small,
                             **W.constant_T(0.5, 200)),
    }


EDGE = _edge_cases()


@pytest.mark.parametrize("name", sorted(EDGE))
@pytest.mark.parametrize("prec", [F64, F32])
def test_edge_cases(ctx, name, prec):
    cfg = EDGE[name]
    ref = oracle.run(cfg, want_psi=True, jump_log_cap=JLOG)
    out = gpu_run(ctx, cfg, prec, jump_log_cap=JLOG)
    st = compare(ref, out, prec, label=name)
    print(name, prec, st)
    if name == "rmax":
        assert (out["status"] == qt.QT_TRAJ_RMAX).any() and (out["status"] == qt.QT_TRAJ_OK).any()
    if name == "maxjumps_1":
        assert (out["status"] == qt.QT_TRAJ_MAXJUMPS).any()
    if name == "zero_steps":
        assert np.all(out["steps_done"] == 0)


@pytest.mark.parametrize("name", ["ragged_3", "deriv1_gamma_bjorken", "rmax", "maxjumps_1"])
def test_edge_cases_plain(ctx, name):
    cfg = EDGE[name]
    ref = oracle.run(cfg, want_psi=True, jump_log_cap=JLOG)
    out = gpu_run(ctx, cfg, F64, PLAIN, jump_log_cap=JLOG)
    compare(ref, out, F64, label="plain " + name)


# ------------------------------------------------------ jump sequences

@pytest.mark.parametrize("prec,form", [(F64, FUSED), (F64, PLAIN), (F32, FUSED)])
def test_jump_sequences_match_the_oracle(ctx, prec, form):
    """Many jumps per trajectory (strong width, Bjorken cooling, thermal
    shift): the device jump log, (step, l, colour) of every jump, equals the
    oracle's for every trajectory away from a threshold; near ones are
    counted and their sequences checked for validity.  A short log (cap 3)
    keeps the first three entries and leaves the rest untouched."""
    tau, T = W.bjorken_table(0.5, 0.6, 0.25, 400)
    cfg = W.base(N=256, L=20.0, dt=0.001, kappa_hat=30.0, gamma_hat=-1.0, n_traj=24, seed=31,
                 init_kind=W.INIT_GAUSSIAN, init_width=1.0, tau=tau, T=T,
                 tau_start=float(tau[0]), T_final=0.25, max_steps=800)
    ref = oracle.run(cfg, want_psi=True, jump_log_cap=JLOG)
    out = gpu_run(ctx, cfg, prec, form, jump_log_cap=JLOG)
    st = compare(ref, out, prec, label="jump log")
    print("jump log", prec, form, st, "jumps", int(ref["n_jumps"].sum()))
    assert int(ref["n_jumps"].sum()) >= 40 and st["jumps_logged"] >= 30
    short = gpu_run(ctx, cfg, prec, form, want_psi=False, jump_log_cap=3)
    for i in range(cfg["n_traj"]):
        k = min(3, int(short["n_jumps"][i]))
        np.testing.assert_array_equal(short["jump_log"][i, :k], out["jump_log"][i, :k])
        assert np.all(short["jump_log"][i, k:] == -1)


def test_empty_batch(ctx):
    cfg = W.base(N=256, n_traj=0, **W.constant_T(0.5, 10))
    out = gpu_run(ctx, cfg, F64)
    assert len(out["norm"]) == 0
    out = gpu_run(ctx, cfg, F64, PLAIN)
    assert len(out["norm"]) == 0


# ----------------------------------------------------------- every grid size

@pytest.mark.parametrize("N", [256, 512, 1024, 2048, 4096, 8192])
@pytest.mark.parametrize("prec", [F64, F32])
def test_grid_sizes(ctx, N, prec):
    steps = {256: 200, 512: 150, 1024: 100, 2048: 60, 4096: 30, 8192: 12}[N]
    cfg = W.base(N=N, L=N * 5.0 / 256.0, dt=0.001, kappa_hat=50.0, n_traj=2, seed=13,
                 init_kind=W.INIT_GAUSSIAN, init_width=1.0, init_l=1, **W.constant_T(0.5, steps))
    ref = oracle.run(cfg, want_psi=True)
    out = gpu_run(ctx, cfg, prec)
    print(N, prec, compare(ref, out, prec, label="N=%d" % N))


# ----------------------------------------- FP32 over the full batch length

def test_fp32_over_the_full_length_against_fp64(ctx):
    """FP32-bulk against fused FP64 (itself within ~1e-12 of the oracle, which
    is too slow for this length) over all 11,899 steps of the N = 2048 batch,
    512 trajectories of the kappa_hat = 1, gamma_hat = -2 run.  Every jump
    history (count, l, colour, status) is the same.  A trajectory whose norm
    passes close to a threshold may jump one step apart in the two
    precisions (a discontinuous decision); the others, which never come
    within 1e-4 of one, agree in wave function and norm to 1e-4 and in the
    overlaps to 5e-5 (measured 5.3e-5, 5.5e-5 and 2.5e-5)."""
    cfg = W.c2_headline(1.0, -2.0, n_traj=512)
    a = gpu_run(ctx, cfg, F64, want_psi=True)
    b = gpu_run(ctx, cfg, F32, want_psi=True)
    assert int(a["steps_done"].max()) == 11899
    for key in ("n_jumps", "l", "color", "status", "steps_done"):
        np.testing.assert_array_equal(a[key], b[key], err_msg=key)
    far = np.minimum(a["min_gap"], b["min_gap"]) > 1e-4
    assert far.sum() >= 50
    da = np.linalg.norm((a["psi"][far] - b["psi"][far]).reshape(far.sum(), -1), axis=1)
    na = np.linalg.norm(a["psi"][far].reshape(far.sum(), -1), axis=1)
    e = dict(far=int(far.sum()), psi=float((da / na).max()),
             norm=float((np.abs(a["norm"][far] - b["norm"][far]) / a["norm"][far]).max()),
             overlap=float(np.abs(a["overlap"][far] - b["overlap"][far]).max()),
             survival=float(np.abs(a["survival"][far] - b["survival"][far]).max()))
    print("fp32 full length", e)
    assert e["psi"] <= 1e-4 and e["norm"] <= 1e-4 and e["overlap"] <= 5e-5


# ------------------------------------------------- every kernel variant

@pytest.mark.parametrize("N", [256, 512, 1024, 2048, 4096, 8192])
def test_every_kernel_variant(N):
    """Each fused kernel variant (threads per trajectory) of each precision,
    fixed with qt_plan_set, and the KSU kernel of this N, against the oracle:
    the tuner may pick any of them (the benchmark runs the tuned ones)."""
    steps = {256: 120, 512: 100, 1024: 80, 2048: 50, 4096: 24, 8192: 10}[N]
    cfg = W.base(N=N, L=N * 5.0 / 256.0, dt=0.001, kappa_hat=50.0, n_traj=2, seed=21,
                 init_kind=W.INIT_GAUSSIAN, init_width=1.0, init_l=1, **W.constant_T(0.5, steps))
    ref = oracle.run(cfg, want_psi=True)
    tau, T = W.bjorken_table(0.5, 0.6, 0.2, 50)
    ksu = W.base(N=N, L=N * 5.0 / 256.0, dt=0.002, potential=W.POTENTIAL_KSU, md_factor=1.2,
                 do_jumps=0, kappa_hat=0.0, n_traj=2, seed=22, tau=tau, T=T,
                 tau_start=float(tau[0]), T_final=0.2, max_steps=steps,
                 init_kind=W.INIT_GAUSSIAN, init_l=0, init_width=2.0)
    ref_ksu = oracle.run(ksu, want_psi=True)
    for prec in (F64, F32):
        variants = qt.plan_variants(N, prec)
        assert variants
        for w in variants:
            c = qt.Context(0)
            try:
                c.plan_set(N, prec, w)
                assert c.plan(N, prec)[0] == w
                out = gpu_run(c, cfg, prec)
                print("variant", N, prec, w, compare(ref, out, prec, label="N=%d W=%d" % (N, w)))
            finally:
                c.close()
        c = qt.Context(0)
        try:
            out = gpu_run(c, ksu, prec)
            print("ksu variant", N, prec, compare(ref_ksu, out, prec, label="ksu N=%d" % N))
        finally:
            c.close()
    with pytest.raises(qt.QtError):
        c = qt.Context(0)
        try:
            c.plan_set(N, F32, 7)
        finally:
            c.close()


# ------------------------------------- C2 at full size, sampled trajectories

C2_SAMPLE = [0, 1, 2047, 4095]


# Trajectories per CU of the benchmark's variants: the three-wave forms
# (LDS and 168 registers sized for three waves per SIMD) and a two-wave one.
# A change that grows their LDS or registers past the budget would cost a
# third of the resident trajectories without failing any other test.
@pytest.mark.parametrize("N,prec,w,per_cu", [(2048, F32, 128, 6), (4096, F32, 256, 3),
                                            (2048, F64, 256, 3), (1024, F64, 128, 6),
                                            (1024, F32, 64, 8)])
def test_forms_keep_their_occupancy(N, prec, w, per_cu):
    c = qt.Context(0)
    try:
        c.plan_set(N, prec, w)
        assert c.plan(N, prec) == (w, per_cu)
    finally:
        c.close()


@pytest.mark.parametrize("prec,form", [(F64, FUSED), (F32, FUSED), (F64, PLAIN)])
def test_c2_full_batch_sampled(ctx, prec, form):
    """4096 trajectories at N=2048 in the benchmark's launch configuration,
    truncated to 120 steps; sampled trajectories against the oracle, every
    trajectory against the invariants."""
    cfg = W.c2_headline(kappa_hat=4.0, gamma_hat=-2.0)
    cfg["max_steps"] = 120
    if form == FUSED:
        ctx.plan(2048, prec, tune=True)     # the variant the benchmark runs
    out = gpu_run(ctx, cfg, prec, form, want_psi=False)
    assert np.all(out["steps_done"] == 120) or np.all(out["status"] != qt.QT_TRAJ_OK)
    assert np.all((out["norm"] > 0) & (out["norm"] <= 1.0 + 1e-6))
    assert np.all((out["l"] - cfg["init_l"] - out["n_jumps"]) % 2 == 0)   # each jump: l +- 1
    assert np.all(out["color"][out["n_jumps"] == 0] == W.SINGLET)
    assert np.all(out["color"][out["n_jumps"] == 1] == W.OCTET)
    for tid in C2_SAMPLE:
        ref = oracle.run(cfg, n_traj=1, traj_id0=tid)
        one = {k: v[tid:tid + 1] for k, v in out.items()}
        compare(ref, one, prec, check_psi=False, label="c2 id %d" % tid)


def test_determinism(ctx):
    cfg = W.c1_parity()
    a = gpu_run(ctx, cfg, F32)
    b = gpu_run(ctx, cfg, F32)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


# ------------------------------------------------ unitarity with kappa = 0

# FP64: every step multiplies by unit-modulus factors (static phase, thermal
# phase, kinetic factor, FFT twiddles) whose moduli are 1 only to an ulp, and
# the same factors recur step after step, so their rounding adds up: a few
# 1e-16 per factor and step, ~1e-12 after 1000 steps (measured 2.9e-12; the
# oracle's naive transform, with fewer factors, 3e-13).  FP32-bulk
# renormalises the unitary block every step.
@pytest.mark.parametrize("prec,tol", [(F64, 1e-11), (F32, 1e-5)])
def test_unitary_evolution_keeps_the_norm(ctx, prec, tol):
    """Without the imaginary potential every sub-step is unitary: after 1000
    steps (thermal shift on, Bjorken cooling, l = 1 octet included) the norm
    stays 1 to rounding; the oracle agrees."""
    tau, T = W.bjorken_table(0.45, 0.6, 0.25, 500)
    cfg = W.base(N=1024, L=20.0, dt=0.001, kappa_hat=0.0, gamma_hat=-2.0, do_jumps=0,
                 tau=tau, T=T, tau_start=float(tau[0]), T_final=0.25, max_steps=1000,
                 init_kind=W.INIT_GAUSSIAN, init_l=1, init_color=W.OCTET, init_width=1.0,
                 n_traj=3, seed=7)
    out = gpu_run(ctx, cfg, prec)
    drift = float(np.max(np.abs(out["norm"] - 1.0)))
    print("norm drift", prec, drift)
    assert np.all(out["steps_done"] == 1000)
    assert drift <= tol
    ref = oracle.run(cfg, n_traj=1)
    assert abs(ref["norm"][0] - 1.0) <= 1e-12


# ------------------------------------------------ kappa_hat(T) lattice fits

@pytest.mark.parametrize("fit", [-1.0, -2.0, -3.0])
@pytest.mark.parametrize("prec,form", [(F64, FUSED), (F64, PLAIN), (F32, FUSED)])
def test_kappa_fit_against_oracle(ctx, fit, prec, form):
    """kappa_hat(T) from the central/lower/upper fit, along a cooling
    Bjorken table, with jumps: every trajectory matches the oracle."""
    tau, T = W.bjorken_table(0.5, 0.6, 0.25, 300)
    cfg = W.base(N=512, L=20.0, dt=0.002, kappa_hat=fit, gamma_hat=-1.5, n_traj=10, seed=21,
                 init_kind=W.INIT_GAUSSIAN, init_width=1.5, tau=tau, T=T,
                 tau_start=float(tau[0]), T_final=0.25, max_steps=600)
    ref = oracle.run(cfg, want_psi=True)
    out = gpu_run(ctx, cfg, prec, form=form)
    print("kappa fit", fit, prec, form, compare(ref, out, prec, label="kappa fit"),
          "jumps", int(ref["n_jumps"].sum()))


# --------------------------------------------------- isotropic KSU potential

@pytest.mark.parametrize("prec,form", [(F64, FUSED), (F64, PLAIN), (F32, FUSED)])
def test_ksu_potential_against_oracle(ctx, prec, form):
    """The isotropic KSU potential (singlet, no jumps) along a Bjorken
    cooling from 0.5 GeV, Coulomb 1S and Gaussian l = 1 starts: every
    trajectory matches the oracle."""
    tau, T = W.bjorken_table(0.5, 0.6, 0.2, 300)
    for init in (dict(init_kind=W.INIT_COULOMB), dict(init_kind=W.INIT_GAUSSIAN, init_l=1,
                                                      init_width=2.0)):
        cfg = W.base(N=512, L=20.0, dt=0.002, potential=W.POTENTIAL_KSU, md_factor=1.2,
                     do_jumps=0, kappa_hat=0.0, n_traj=3, seed=8, tau=tau, T=T,
                     tau_start=float(tau[0]), T_final=0.2, max_steps=700, **init)
        ref = oracle.run(cfg, want_psi=True)
        out = gpu_run(ctx, cfg, prec, form=form)
        print("ksu", prec, form, init["init_kind"], compare(ref, out, prec, label="ksu"),
              "norm", float(ref["norm"][0]))
        assert ref["norm"][0] < 0.999          # the width acted


def test_ksu_rejects_jumps_and_octet(ctx):
    cfg = W.base(N=512, L=20.0, potential=W.POTENTIAL_KSU, n_traj=2, **W.constant_T(0.3, 10))
    with pytest.raises(qt.QtError):
        gpu_run(ctx, cfg, F64)                                   # do_jumps = 1
    with pytest.raises(qt.QtError):
        gpu_run(ctx, dict(cfg, do_jumps=0, init_color=W.OCTET, init_kind=W.INIT_GAUSSIAN,
                          init_width=1.0), F64)


# ------------------------------- the N = 2048 batch over its whole length

def _c2_goldens():
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "c2_full_length_oracle.json")
    return json.load(open(path))["rows"]


@pytest.mark.parametrize("form", [FUSED, PLAIN])
def test_fp64_full_length_against_oracle_goldens(ctx, form):
    """FP64 over all 11,899 steps of the N = 2048 Bjorken batch, two
    trajectories of each (kappa_hat, gamma_hat) run, against the oracle's
    results stored by tests/golden/make_c2_full_length.py: every result and
    the whole jump sequence, to the FP64 bar (1e-10)."""
    rows = _c2_goldens()
    for run in sorted({(r["kappa_hat"], r["gamma_hat"]) for r in rows}):
        cfg = W.c2_headline(*run)
        for r in [x for x in rows if (x["kappa_hat"], x["gamma_hat"]) == run]:
            out = gpu_run(ctx, cfg, F64, form, want_psi=False, n_traj=1, traj_id0=r["traj_id"],
                          jump_log_cap=64)
            assert r["min_gap"] > FP64_DELTA                 # decisions well away from 1e-9
            for key in ("status", "steps_done", "n_jumps", "l", "color"):
                assert out[key][0] == r[key], (run, r["traj_id"], key)
            assert out["steps_done"][0] == r["n_steps"] == 11899
            np.testing.assert_array_equal(out["jump_log"][0, :len(r["jump_log"])],
                                          np.array(r["jump_log"], dtype=np.int32).reshape(-1, 3))
            assert out["first_r"][0] == r["first_r"]
            assert abs(out["norm"][0] - r["norm"]) <= 1e-10
            assert np.max(np.abs(out["overlap"][0] - r["overlap"])) <= 1e-10
            assert np.max(np.abs(out["survival"][0] - r["survival"])) <= 1e-10
            assert abs(out["mean_r"][0] - r["mean_r"]) <= 1e-9 * r["mean_r"]
