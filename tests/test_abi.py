"""The C-ABI library loads and exports every function include/qtraj.h
declares (no GPU needed: nothing here launches a kernel)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qtraj.h")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:qt_status|const char\*)\s+(qt_\w+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def qtlib():
    from paper_2107_06147_amd import qtraj
    if not os.path.exists(qtraj.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return qtraj


def test_header_declares_the_api():
    names = declared()
    assert "qt_run" in names and "qt_submit" in names and len(names) >= 20


def test_every_declared_symbol_is_exported(qtlib):
    lib = ctypes.CDLL(qtlib.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding wraps exactly those
    assert sorted(qtlib.SYMBOLS) == declared()


def test_version_and_error_without_gpu(qtlib):
    L = qtlib.lib()
    assert b"gfx950" in L.qt_version()
    assert isinstance(L.qt_last_error(), bytes)
    # a null context is rejected without touching the device
    assert L.qt_run(None, None, None, None, None, None, None) == qtlib.QT_EINVAL
    assert b"null" in L.qt_last_error()


def test_oracle_and_library_share_no_code():
    """The GPU library's sources never include or name the oracle, and the
    oracle never includes the library's headers."""
    csrc = os.path.join(ROOT, "paper_2107_06147_amd", "csrc")
    for f in os.listdir(csrc):
        txt = open(os.path.join(csrc, f)).read()
        assert "oracle" not in txt.lower(), f
    for f in ("qtraj_oracle.c", "qtraj_oracle.h"):
        txt = open(os.path.join(ROOT, "oracle", f)).read()
        assert "qtraj.h" not in txt and "qt_internal" not in txt and "csrc" not in txt
    for f in ("qtraj.py", "__init__.py", "build.py"):
        txt = open(os.path.join(ROOT, "paper_2107_06147_amd", f)).read()
        assert "import oracle" not in txt and "from oracle" not in txt, f


def test_count_steps_matches_the_stepwise_definition(qtlib):
    """qt_count_steps (host only) passes whole intervals of the table at once
    where T cannot cross T_final; the oracle takes every step.  The two agree
    on Bjorken and random-walk (non-monotone) tables, starts before, inside
    and at the table's points, steps that land exactly on points, T_final
    equal to a point's T, and step caps."""
    import numpy as np
    import oracle
    from paper_2107_06147_amd import workloads as W
    rng = np.random.default_rng(7)
    cases = 0
    for trial in range(300):
        kind = trial % 4
        dt = float(rng.choice([0.001, 0.0005, 0.0123, 0.25, 0.5]))
        if kind == 0:
            tau, T = W.bjorken_table(float(rng.uniform(0.3, 0.55)), float(rng.uniform(0.4, 0.8)), 0.25,
                                     int(rng.integers(2, 60)))
            tf = float(rng.choice([0.25, 0.3, 0.0, float(T[len(T) // 2])]))
        elif kind == 1:
            tau, T = W.random_walk_table(rng, n_points=int(rng.integers(5, 80)))
            tf = float(rng.choice([0.3, 0.4, float(T[int(rng.integers(len(T)))])]))
        elif kind == 2:
            # points on multiples of dt: steps land exactly on them
            k = np.cumsum(rng.integers(1, 6, size=int(rng.integers(2, 12))))
            tau = (k - k[0]).astype(float) * dt
            T = rng.choice([0.2, 0.3, 0.4], size=len(tau)).astype(float)
            tf = float(rng.choice([0.2, 0.3, 0.4]))
        else:
            tau = np.sort(rng.uniform(0.0, 50.0, size=int(rng.integers(2, 30))))
            tau = np.unique(tau)
            if len(tau) < 2:
                continue
            T = rng.uniform(0.0, 1.0, size=len(tau))
            tf = float(rng.uniform(0.0, 0.5))
        span = float(tau[-1] - tau[0])
        start = float(rng.choice([tau[0], tau[0] - 3.5 * dt, tau[0] + 0.3 * span,
                                  float(tau[len(tau) // 2]), tau[-1]]))
        cap = int(rng.choice([0, 1, 7, 1000, 2 ** 62]))
        cfg = W.base(N=256, dt=dt, tau=np.asarray(tau, float), T=np.asarray(T, float),
                     tau_start=start, T_final=tf, max_steps=cap)
        assert qtlib.count_steps(cfg) == oracle.num_steps(cfg), (trial, kind, dt, start, tf, cap)
        cases += 1
    assert cases > 250
    # an invalid table is rejected, as qt_run rejects it
    bad = W.base(N=256, dt=0.001, tau=np.array([0.0, 0.0]), T=np.array([0.3, 0.3]),
                 tau_start=0.0, T_final=0.0, max_steps=10)
    with pytest.raises(RuntimeError):
        qtlib.count_steps(bad)


def test_plan_variants_host_query(qtlib):
    """The fused kernel variants are listed without a device; every N from
    256 to 8192 has at least one in each precision."""
    for N in (256, 512, 1024, 2048, 4096, 8192):
        for prec in (qtlib.QT_FP64, qtlib.QT_FP32_BULK):
            ws = qtlib.plan_variants(N, prec)
            assert ws and ws == sorted(ws) and all(w % 64 == 0 and N % w == 0 for w in ws), (N, prec, ws)
    assert 128 in qtlib.plan_variants(2048, qtlib.QT_FP32_BULK)
    assert qtlib.plan_variants(3000, qtlib.QT_FP64) == []
    L = qtlib.lib()
    assert L.qt_plan_variants(2048, 0, None, 0, None) == qtlib.QT_EINVAL


def test_results_pointer_table_matches_per_batch_structs(qtlib):
    """run_many's flat results: the pointer table built at once equals the
    qt_results built batch by batch (host tensors; nothing is launched)."""
    import torch
    counts = [3, 1, 7, 2]
    total = sum(counts)
    out = {n: torch.zeros(total, dtype=torch.float64) for n in ("norm", "first_r", "mean_r", "min_gap")}
    out["overlap"] = torch.zeros(total, 6, dtype=torch.float64)
    out["survival"] = torch.zeros(total, 6, dtype=torch.float64)
    for n in ("l", "color", "n_jumps", "status"):
        out[n] = torch.zeros(total, dtype=torch.int32)
    out["steps_done"] = torch.zeros(total, dtype=torch.int64)
    rows = [0, 3, 4, 11]
    keep = []
    arr = qtlib.results_array(out, rows, keep)
    for i, row in enumerate(rows):
        one = qtlib.results_struct(out, row)
        for f in qtlib._RESULT_FIELDS:
            a = ctypes.cast(getattr(arr[i], f), ctypes.c_void_p).value
            b = ctypes.cast(getattr(one, f), ctypes.c_void_p).value
            assert a == b, (i, f)
    assert ctypes.cast(arr[2].psi, ctypes.c_void_p).value is None      # no wave functions: null
