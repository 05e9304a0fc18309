"""Segmented runs (checkpoints, HIP-graph replay, save/restore), uneven
batches in one job, and the continuous-batching server.  Marked `gpu`."""
import numpy as np
import pytest

import oracle
from paper_2107_06147_amd import qtraj as qt
from paper_2107_06147_amd import workloads as W
from tests.gpu_parity import compare, gpu_run

pytestmark = pytest.mark.gpu

F64, F32 = qt.QT_FP64, qt.QT_FP32_BULK
KEYS = ("norm", "first_r", "overlap", "survival", "mean_r", "l", "color", "n_jumps", "status",
        "steps_done", "min_gap")


@pytest.fixture(scope="module")
def ctx():
    c = qt.Context(0)
    yield c
    c.close()


def _cfg(N=512, steps=300):
    return W.base(N=N, L=N * 20.0 / 512, dt=0.001, kappa_hat=20.0, n_traj=40, seed=17,
                  init_kind=W.INIT_GAUSSIAN, init_width=1.0, **W.constant_T(0.5, steps))


def _same(a, b, keys=KEYS + ("psi",)):
    for k in keys:
        if k in a and k in b:
            assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k


@pytest.mark.parametrize("N,steps", [(512, 300), (2048, 120)])
@pytest.mark.parametrize("prec", [F32, F64])
def test_segments_equal_single_run(ctx, prec, N, steps):
    """Also at N = 2048, where workgroups of several waves keep the static
    phase cached across steps (filled again after each jump and at each
    resumed segment)."""
    import torch
    cfg = _cfg(N, steps)
    ref = gpu_run(ctx, cfg, prec)
    assert ref["n_jumps"].sum() > 0
    job = qt.Job(ctx, cfg, precision=prec, segment_steps=37)
    job.advance(steps)
    assert job.done()
    out = qt.to_numpy(job.results(want_psi=True))
    torch.cuda.synchronize()
    job.close()
    _same(ref, out)


def test_graph_replay_and_checkpoint_resume(ctx):
    import torch
    cfg = _cfg()
    ref = gpu_run(ctx, cfg, F32)
    a = qt.Job(ctx, cfg, precision=F32, segment_steps=25)
    for _ in range(3):                     # the same captured graph, three times
        a.advance(50)
    assert not a.done()
    blob = torch.empty(a.state_bytes(), dtype=torch.uint8)        # host checkpoint
    a.save(blob.data_ptr())
    torch.cuda.synchronize()
    a.close()
    b = qt.Job(ctx, cfg, precision=F32, segment_steps=25)
    b.load(blob.data_ptr())
    b.advance(150)
    assert b.done()
    out = qt.to_numpy(b.results(want_psi=True))
    torch.cuda.synchronize()
    b.close()
    _same(ref, out)


def _job_steps(job, n):
    """(step, done) of every trajectory, read from a host checkpoint (the
    88-byte state records lead the blob: step int64 at offset 0, done int32
    at offset 28)."""
    import torch
    blob = torch.empty(job.state_bytes(), dtype=torch.uint8)
    job.save(blob.data_ptr())
    torch.cuda.synchronize()
    rec = blob.numpy()[:88 * n].reshape(n, 88)
    return rec[:, 0:8].copy().view(np.int64)[:, 0], rec[:, 28:32].copy().view(np.int32)[:, 0]


@pytest.mark.parametrize("prec", [F32, F64])
def test_advance_takes_exactly_the_steps_asked(ctx, prec):
    """advance(50) with segments of 37 steps runs 50 steps (a segment of 37,
    then one of 13), advance(10) with segments of 1000 runs 10; every
    unfinished trajectory's checkpoint is at that step, and the finished
    run equals a single one."""
    import torch
    cfg = dict(_cfg(512, 300), kappa_hat=2.0)
    ref = gpu_run(ctx, cfg, prec)
    job = qt.Job(ctx, cfg, precision=prec, segment_steps=37)
    job.advance(50)
    step, done = _job_steps(job, cfg["n_traj"])
    assert np.all(step[done == 0] == 50) and (done == 0).sum() > 0
    job.advance(50)                            # the same graph again
    step, done = _job_steps(job, cfg["n_traj"])
    assert np.all(step[done == 0] == 100)
    job.advance(200)
    assert job.done()
    _same(ref, qt.to_numpy(job.results(want_psi=True)))
    torch.cuda.synchronize()
    job.close()
    job = qt.Job(ctx, cfg, precision=prec, segment_steps=1000)
    job.advance(10)
    step, done = _job_steps(job, cfg["n_traj"])
    assert np.all(step[done == 0] == 10)
    job.close()


def test_job_fp64_matches_oracle(ctx):
    import torch
    cfg = _cfg()
    ref = oracle.run(cfg, want_psi=True)
    job = qt.Job(ctx, cfg, precision=F64, segment_steps=100)
    job.advance(300)
    out = qt.to_numpy(job.results(want_psi=True))
    torch.cuda.synchronize()
    job.close()
    compare(ref, out, F64, label="job fp64")


def test_run_many_uneven_equals_separate_runs(ctx):
    """Batches of N = 1024/2048/4096 with different lifetimes in one job give
    bitwise the results of separate runs, and match the oracle (FP64)."""
    import torch
    cfgs = W.c3_uneven(n_traj=9)
    for i, c in enumerate(cfgs):
        c["max_steps"] = 40 + 30 * i          # uneven lifetimes
        c["n_traj"] = 2
    outs = qt.run_many(ctx, cfgs, precision=F64, want_psi=True)
    torch.cuda.synchronize()
    for c, o in zip(cfgs, outs):
        alone = gpu_run(ctx, c, F64)
        _same(alone, qt.to_numpy(o))
    for c, o in list(zip(cfgs, outs))[:3]:
        compare(oracle.run(c, want_psi=True), qt.to_numpy(o), F64, label="many N=%d" % c["N"])


def test_run_many_flat_equals_per_batch(ctx):
    """flat=True puts every batch's results one after the other in one set of
    tensors, equal to the per-batch results; batches that share N and L
    share their tables on the device."""
    import torch
    cfgs = W.c3_uneven(n_traj=12)
    for i, c in enumerate(cfgs):
        c["max_steps"] = 25 + 7 * i
        c["n_traj"] = 1 + (i % 3)
    per = qt.run_many(ctx, cfgs, precision=F32)
    flat = qt.run_many(ctx, cfgs, precision=F32, flat=True)
    torch.cuda.synchronize()
    row = 0
    for c, o in zip(cfgs, per):
        n = int(c["n_traj"])
        a = qt.to_numpy(o)
        b = {k: v[row:row + n] for k, v in qt.to_numpy(flat).items()}
        row += n
        _same(a, b)
    assert row == len(flat["norm"])


# ------------------------------------------------------------------ server --

def _requests():
    tau, T = W.random_walk_table(np.random.default_rng(5))
    r1 = W.base(N=1024, L=20.0, dt=0.001, kappa_hat=4.0, n_traj=30, seed=101,
                init_kind=W.INIT_GAUSSIAN, init_width=1.0, tau=tau, T=T, tau_start=float(tau[0]),
                T_final=0.0, max_steps=200)
    r2 = W.base(N=2048, L=40.0, dt=0.001, kappa_hat=8.0, n_traj=20, seed=102,
                init_kind=W.INIT_GAUSSIAN, init_width=1.0, **W.constant_T(0.45, 150))
    r3 = W.base(N=1024, L=20.0, dt=0.001, kappa_hat=4.0, gamma_hat=-2.0, n_traj=25, seed=103,
                init_kind=W.INIT_COULOMB, **W.constant_T(0.35, 260))
    return [r1, r2, r3]


def test_server_alone_vs_mix_bitwise(ctx):
    """Each request's result in the concurrent mix equals its result alone,
    bit for bit, and the oracle's within the FP32-bulk bounds."""
    reqs = _requests()
    alone = [gpu_run(ctx, c, F32) for c in reqs]
    srv = qt.Server(ctx, precision=F32, segment_steps=64)
    ids = [srv.submit(c) for c in reqs]
    outs = [srv.wait(i, timeout_s=120, want_psi=True) for i in ids]
    st = srv.stats()
    srv.close()
    for a, o in zip(alone, outs):
        _same(a, o)
    assert st["completed"] == 3 and st["p99_latency_s"] >= st["p50_latency_s"] > 0
    assert st["traj_steps"] == sum(int(a["steps_done"].sum()) for a in alone)
    for c, o in zip(reqs, outs):
        print("server vs oracle", c["N"], compare(oracle.run(c, want_psi=True), o, F32,
                                                  label="server N=%d" % c["N"]))


def test_server_admission_failure_has_its_own_status(ctx):
    """A request that passes the budget but whose state does not fit the
    device (655 GB of wave functions) fails at admission with QT_ENOMEM, not
    as a cancellation; the server goes on with the next request."""
    srv = qt.Server(ctx, precision=F32, segment_steps=50, hbm_budget_bytes=1 << 50)
    big = dict(_requests()[0], N=8192, L=160.0, n_traj=10_000_000, max_steps=10)
    rid = srv.submit(big)
    with pytest.raises(qt.QtError) as e:
        srv.wait(rid, timeout_s=120)
    assert e.value.status == qt.QT_ENOMEM
    good = _requests()[0]
    out = srv.wait(srv.submit(good), timeout_s=120)
    assert np.all(out["steps_done"] == 200)
    srv.close()


def test_server_rejects_bad_requests_and_keeps_running(ctx):
    srv = qt.Server(ctx, precision=F32, segment_steps=50, hbm_budget_bytes=64 << 20)
    good = _requests()[0]
    rid = srv.submit(good)
    bad = dict(good, N=300)
    with pytest.raises(qt.QtError) as e:
        srv.submit(bad)
    assert e.value.status == qt.QT_EINVAL
    huge = dict(good, N=4096, L=80.0, n_traj=200000)
    with pytest.raises(qt.QtError) as e:
        srv.submit(huge)
    assert e.value.status == qt.QT_ENOMEM
    long = dict(good, max_steps=100000)
    rid2 = srv.submit(long)
    srv.cancel(rid2)
    out = srv.wait(rid, timeout_s=120)
    assert np.all(out["steps_done"] == 200)
    with pytest.raises(qt.QtError) as e:
        srv.wait(rid2, timeout_s=120)
    assert e.value.status == qt.QT_ECANCELED
    srv.close()


def test_eigen_basis_and_ksu_through_jobs_and_server(ctx):
    """Segmented jobs and the server reproduce single runs bitwise for the
    computed eigenstate basis (initType 100 with ProjType 1) and for the
    KSU potential."""
    import torch
    tau, T = W.bjorken_table(0.5, 0.6, 0.25, 200)
    eig = W.base(N=512, L=20.0, dt=0.001, kappa_hat=4.0, n_traj=12, seed=41,
                 init_kind=W.INIT_EIGEN, init_n=1, init_l=0, basis=W.BASIS_EIGEN,
                 **W.constant_T(0.45, 250))
    ksu = W.base(N=512, L=20.0, dt=0.002, potential=W.POTENTIAL_KSU, do_jumps=0,
                 kappa_hat=0.0, n_traj=6, seed=42, tau=tau, T=T, tau_start=float(tau[0]),
                 T_final=0.25, max_steps=250)
    for cfg in (eig, ksu):
        ref = gpu_run(ctx, cfg, F32)
        job = qt.Job(ctx, cfg, precision=F32, segment_steps=40)
        job.advance(250)
        assert job.done()
        out = qt.to_numpy(job.results(want_psi=True))
        torch.cuda.synchronize()
        job.close()
        _same(ref, out)
    srv = qt.Server(ctx, precision=F32, segment_steps=64)
    ids = [srv.submit(c) for c in (eig, ksu)]
    outs = [srv.wait(i, timeout_s=120, want_psi=True) for i in ids]
    srv.close()
    for c, o in zip((eig, ksu), outs):
        _same(gpu_run(ctx, c, F32), o)


def test_c5_full_batch_sampled(ctx):
    """The N = 4096 batch of 65,536 trajectories (three initial states) in
    the benchmark's configuration (tuned variant, segmented jobs replayed as
    HIP graphs), truncated to 40 steps: every trajectory against the
    invariants, the first and last of each initial state against the
    oracle."""
    import torch
    cfgs = W.c5_roofline(n_steps=40)
    assert sum(int(c["n_traj"]) for c in cfgs) == 65536
    ctx.plan(4096, F32, tune=True)
    jobs = [qt.Job(ctx, c, precision=F32, segment_steps=20) for c in cfgs]
    for j in jobs:
        j.advance(40)
    outs = [qt.to_numpy(j.results()) for j in jobs]
    torch.cuda.synchronize()
    for j in jobs:
        j.close()
    for cfg, out in zip(cfgs, outs):
        assert np.all(out["steps_done"] == 40)
        assert np.all((out["norm"] > 0) & (out["norm"] <= 1.0 + 1e-6))
        assert np.all((out["l"] - cfg["init_l"] - out["n_jumps"]) % 2 == 0)
        for k in (0, int(cfg["n_traj"]) - 1):
            tid = int(cfg["traj_id0"]) + 3 * k
            ref = oracle.run(cfg, n_traj=1, traj_id0=tid)
            one = {key: v[k:k + 1] for key, v in out.items()}
            compare(ref, one, F32, check_psi=False, label="c5 id %d" % tid)



def test_trace_lines(ctx, tmp_path, monkeypatch):
    """QTRAJ_TRACE names a file: a run, a job segment and a server round each
    append one JSON line with their sizes and device time."""
    import json
    path = tmp_path / "trace.jsonl"
    monkeypatch.setenv("QTRAJ_TRACE", str(path))
    cfg = _cfg(512, 60)
    gpu_run(ctx, cfg, F32)
    job = qt.Job(ctx, cfg, precision=F32, segment_steps=25)
    job.advance(50)
    job.done()
    job.close()
    srv = qt.Server(ctx, precision=F32, segment_steps=100)
    srv.wait(srv.submit(_requests()[0]), timeout_s=120)
    srv.close()
    monkeypatch.delenv("QTRAJ_TRACE")
    lines = [json.loads(x) for x in open(path)]
    ev = {x["event"]: x for x in lines}
    assert {"run", "segment", "round"} <= set(ev)
    assert ev["run"]["items"] == cfg["n_traj"] and ev["run"]["N_classes"] == [512]
    assert ev["run"]["kernel_ms"] > 0
    assert ev["segment"]["steps"] == 50 and ev["segment"]["launches"] == 2
    assert ev["round"]["traj_steps"] > 0
