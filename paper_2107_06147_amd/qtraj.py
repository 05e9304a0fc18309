"""ctypes binding of libqtraj.so (the C ABI of include/qtraj.h).

Argument marshalling only: every step of the solver runs in the library's
HIP kernels.  The functions keep the C names (qt_context_create, qt_run,
...); `run()` and `run_many()` additionally turn the config dicts of
`paper_2107_06147_amd.workloads` into the C structs and allocate the output
tensors on the GPU with torch (torch provides device memory and streams).

If libqtraj.so has not been built this module raises on first use; there is
no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqtraj.so")

QT_OK, QT_EINVAL, QT_ENOMEM, QT_EDEVICE, QT_EBUSY, QT_ETIMEOUT, QT_ECANCELED, QT_ENOTFOUND, QT_ENOCONV = range(9)
QT_FP64, QT_FP32_BULK = 0, 1
QT_FORM_FUSED, QT_FORM_PLAIN = 0, 1
QT_INIT_COULOMB, QT_INIT_GAUSSIAN, QT_INIT_ARRAY, QT_INIT_EIGEN = 0, 1, 2, 3
QT_BASIS_COULOMB, QT_BASIS_EIGEN = 0, 1
QT_SINGLET, QT_OCTET = 0, 1
QT_TRAJ_OK, QT_TRAJ_RMAX, QT_TRAJ_MAXJUMPS, QT_TRAJ_LMAX, QT_TRAJ_NOJUMP = 0, 1, 2, 3, 4
QT_POTENTIAL_MUNICH, QT_POTENTIAL_KSU = 0, 1
QT_FLAG_KINETIC_OFF = 1

_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)
_I64 = C.POINTER(C.c_int64)


class qt_physics(C.Structure):
    _fields_ = [("N", C.c_int32), ("L", C.c_double), ("dt", C.c_double), ("mass", C.c_double),
                ("alpha_s", C.c_double), ("kappa_hat", C.c_double), ("gamma_hat", C.c_double),
                ("deriv_type", C.c_int32), ("do_jumps", C.c_int32), ("max_jumps", C.c_int32),
                ("r_max", C.c_double), ("flags", C.c_int32), ("potential", C.c_int32),
                ("md_factor", C.c_double), ("basis", C.c_int32), ("pad0", C.c_int32)]


class qt_ttable(C.Structure):
    _fields_ = [("tau", _D), ("T", _D), ("n", C.c_int32), ("tau_start", C.c_double),
                ("T_final", C.c_double), ("max_steps", C.c_int64),
                ("vacuum_steps", C.c_int64)]


class qt_init(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32), ("l", C.c_int32), ("color", C.c_int32),
                ("width", C.c_double), ("u_re", _D), ("u_im", _D)]


class qt_batch(C.Structure):
    _fields_ = [("n_traj", C.c_int64), ("seed", C.c_uint64), ("traj_id0", C.c_uint64),
                ("traj_id_stride", C.c_uint64), ("precision", C.c_int32), ("form", C.c_int32),
                ("no_jump_shortcut", C.c_int32)]


class qt_results(C.Structure):
    _fields_ = [("norm", _D), ("first_r", _D), ("overlap", _D), ("survival", _D),
                ("mean_r", _D), ("l", _I32), ("color", _I32), ("n_jumps", _I32),
                ("status", _I32), ("steps_done", _I64), ("min_gap", _D), ("psi", _D),
                ("jump_log", _I32), ("jump_log_cap", C.c_int32), ("pad0", C.c_int32)]


class qt_server_cfg(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("segment_steps", C.c_int64),
                ("precision", C.c_int32), ("pad0", C.c_int32), ("max_occupancy", C.c_double)]


class qt_stats(C.Structure):
    _fields_ = [("p50_latency_s", C.c_double), ("p99_latency_s", C.c_double),
                ("mean_latency_s", C.c_double), ("traj_steps_per_s", C.c_double),
                ("completed", C.c_int64), ("admitted", C.c_int64), ("queued", C.c_int64),
                ("running", C.c_int64), ("traj_steps", C.c_int64), ("hbm_in_use", C.c_size_t)]


# every symbol the header declares, with (restype, argtypes)
_VP = C.c_void_p
_SIGS = {
    "qt_context_create": (C.c_int, [C.c_int, C.POINTER(_VP)]),
    "qt_context_destroy": (C.c_int, [_VP]),
    "qt_run": (C.c_int, [_VP, C.POINTER(qt_physics), C.POINTER(qt_ttable), C.POINTER(qt_init),
                         C.POINTER(qt_batch), C.POINTER(qt_results), _VP]),
    "qt_run_noalloc": (C.c_int, [_VP, C.POINTER(qt_physics), C.POINTER(qt_ttable),
                                 C.POINTER(qt_init), C.POINTER(qt_batch), C.POINTER(qt_results),
                                 _VP]),
    "qt_run_many": (C.c_int, [_VP, C.c_int32, C.POINTER(qt_physics), C.POINTER(qt_ttable),
                              C.POINTER(qt_init), C.POINTER(qt_batch), C.POINTER(qt_results), _VP]),
    "qt_job_create": (C.c_int, [_VP, C.POINTER(qt_physics), C.POINTER(qt_ttable),
                                C.POINTER(qt_init), C.POINTER(qt_batch), C.c_int64,
                                C.POINTER(_VP)]),
    "qt_job_advance": (C.c_int, [_VP, C.c_int64, _VP]),
    "qt_job_done": (C.c_int, [_VP, _I32]),
    "qt_job_state_bytes": (C.c_int, [_VP, C.POINTER(C.c_size_t)]),
    "qt_job_save": (C.c_int, [_VP, _VP, _VP]),
    "qt_job_load": (C.c_int, [_VP, _VP, _VP]),
    "qt_job_results": (C.c_int, [_VP, C.POINTER(qt_results), _VP]),
    "qt_job_destroy": (C.c_int, [_VP]),
    "qt_server_create": (C.c_int, [_VP, C.POINTER(qt_server_cfg), C.POINTER(_VP)]),
    "qt_submit": (C.c_int, [_VP, C.POINTER(qt_physics), C.POINTER(qt_ttable), C.POINTER(qt_init),
                            C.POINTER(qt_batch), C.POINTER(C.c_uint64)]),
    "qt_poll": (C.c_int, [_VP, C.c_uint64, _I32]),
    "qt_wait": (C.c_int, [_VP, C.c_uint64, C.POINTER(qt_results), C.c_double]),
    "qt_cancel": (C.c_int, [_VP, C.c_uint64]),
    "qt_server_stats": (C.c_int, [_VP, C.POINTER(qt_stats)]),
    "qt_server_destroy": (C.c_int, [_VP]),
    "qt_last_kernel_ms": (C.c_int, [_VP, _D, _I64]),
    "qt_plan": (C.c_int, [_VP, C.c_int32, C.c_int32, C.c_int32, _I32, _I32]),
    "qt_eigen_basis": (C.c_int, [_VP, C.POINTER(qt_physics), _D, _D]),
    "qt_count_steps": (C.c_int, [C.POINTER(qt_physics), C.POINTER(qt_ttable), _I64]),
    "qt_plan_variants": (C.c_int, [C.c_int32, C.c_int32, _I32, C.c_int32, _I32]),
    "qt_plan_set": (C.c_int, [_VP, C.c_int32, C.c_int32, C.c_int32]),
    "qt_last_error": (C.c_char_p, []),
    "qt_version": (C.c_char_p, []),
}
SYMBOLS = tuple(_SIGS)

_lib = None


def lib():
    """Load libqtraj.so.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libqtraj.so is missing: build it with __graft_entry__.build() "
                               "(hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class QtError(RuntimeError):
    def __init__(self, status, where):
        msg = lib().qt_last_error().decode(errors="replace")
        super().__init__("%s failed (status %d): %s" % (where, status, msg))
        self.status = status


def check(status, where):
    if status != QT_OK:
        raise QtError(status, where)


# ------------------------------------------------------------ marshalling --

def _dp(a):
    return None if a is None else a.ctypes.data_as(_D)


def physics(cfg):
    return qt_physics(int(cfg["N"]), float(cfg["L"]), float(cfg["dt"]), float(cfg["mass"]),
                      float(cfg["alpha_s"]), float(cfg["kappa_hat"]), float(cfg["gamma_hat"]),
                      int(cfg.get("deriv_type", 0)), int(cfg.get("do_jumps", 1)),
                      int(cfg.get("max_jumps", -1)), float(cfg.get("r_max", 1.0)),
                      int(cfg.get("flags", 0)), int(cfg.get("potential", 0)),
                      float(cfg.get("md_factor", 1.0)), int(cfg.get("basis", 0)), 0)


def ttable(cfg, keep):
    tau = np.ascontiguousarray(cfg["tau"], dtype=np.float64)
    T = np.ascontiguousarray(cfg["T"], dtype=np.float64)
    keep += [tau, T]
    return qt_ttable(_dp(tau), _dp(T), len(tau), float(cfg["tau_start"]),
                     float(cfg.get("T_final", 0.0)), int(cfg.get("max_steps", 2**62)),
                     int(cfg.get("vacuum_steps", 0)))


def init(cfg, keep):
    kind = int(cfg.get("init_kind", QT_INIT_COULOMB))
    u_re = u_im = None
    if kind == QT_INIT_ARRAY:
        u = np.asarray(cfg["u0"])
        u_re = np.ascontiguousarray(u.real, dtype=np.float64)
        u_im = np.ascontiguousarray(u.imag, dtype=np.float64)
        keep += [u_re, u_im]
    return qt_init(kind, int(cfg.get("init_n", 1)), int(cfg.get("init_l", 0)),
                   int(cfg.get("init_color", QT_SINGLET)), float(cfg.get("init_width", 0.0)),
                   _dp(u_re), _dp(u_im))


def batch(cfg, precision, form=QT_FORM_FUSED, n_traj=None, traj_id0=None):
    return qt_batch(int(cfg["n_traj"] if n_traj is None else n_traj), int(cfg.get("seed", 1)),
                    int(cfg.get("traj_id0", 0) if traj_id0 is None else traj_id0),
                    int(cfg.get("traj_id_stride", 1)), int(precision), int(form),
                    int(cfg.get("no_jump_shortcut", 0)))


def alloc_results(n, N, want_psi, device="cuda", jump_log_cap=0):
    """Output tensors on the GPU (torch) and the qt_results of their pointers.
    jump_log_cap > 0 adds a jump log of that many (step, l, colour) entries
    per trajectory, filled with -1 where no jump was logged."""
    import torch
    f64 = dict(dtype=torch.float64, device=device)
    out = {
        "norm": torch.zeros(n, **f64), "first_r": torch.zeros(n, **f64),
        "overlap": torch.zeros(n, 6, **f64), "survival": torch.zeros(n, 6, **f64),
        "mean_r": torch.zeros(n, **f64),
        "l": torch.zeros(n, dtype=torch.int32, device=device),
        "color": torch.zeros(n, dtype=torch.int32, device=device),
        "n_jumps": torch.zeros(n, dtype=torch.int32, device=device),
        "status": torch.zeros(n, dtype=torch.int32, device=device),
        "steps_done": torch.zeros(n, dtype=torch.int64, device=device),
        "min_gap": torch.zeros(n, **f64),
    }
    if want_psi:
        out["psi"] = torch.zeros(n, N, 2, **f64)
    if jump_log_cap > 0:
        out["jump_log"] = torch.full((n, int(jump_log_cap), 3), -1, dtype=torch.int32, device=device)
    return out, results_struct(out)


def results_struct(out, row=0):
    """qt_results of the tensors in `out`, starting at trajectory `row`."""
    def p(name, typ):
        t = out.get(name)
        if t is None:
            return None
        return C.cast(C.c_void_p(t.data_ptr() + row * t.stride(0) * t.element_size()), typ)
    jl = out.get("jump_log")
    return qt_results(p("norm", _D), p("first_r", _D), p("overlap", _D), p("survival", _D),
                      p("mean_r", _D), p("l", _I32), p("color", _I32), p("n_jumps", _I32),
                      p("status", _I32), p("steps_done", _I64), p("min_gap", _D), p("psi", _D),
                      p("jump_log", _I32), 0 if jl is None else int(jl.shape[1]), 0)


# the pointer fields of qt_results (all but the trailing jump_log_cap, pad0)
_RESULT_FIELDS = [f for f, _ in qt_results._fields_][:-2]


def results_array(out, rows, keep):
    """qt_results of the tensors in `out` for every start row in `rows` at
    once (ctypes array; its pointer table is a numpy array kept in `keep`)."""
    rows = np.asarray(rows, dtype=np.int64)
    nf = len(_RESULT_FIELDS)
    base = np.zeros(nf + 1, dtype=np.int64)     # + the (jump_log_cap, pad0) word
    step = np.zeros(nf + 1, dtype=np.int64)
    for j, name in enumerate(_RESULT_FIELDS):
        t = out.get(name)
        if t is not None:
            base[j] = t.data_ptr()
            step[j] = t.stride(0) * t.element_size()
    tab = base[None, :] + rows[:, None] * step[None, :]
    tab[:, base == 0] = 0
    jl = out.get("jump_log")
    tab[:, nf] = 0 if jl is None else int(jl.shape[1])   # little-endian: cap, then pad 0
    tab = np.ascontiguousarray(tab.astype(np.uint64))
    keep.append(tab)
    return (qt_results * len(rows)).from_buffer(tab)


def host_results(n, N, want_psi):
    """Output arrays in host memory (numpy) and their qt_results."""
    out = {
        "norm": np.zeros(n), "first_r": np.zeros(n), "overlap": np.zeros((n, 6)),
        "survival": np.zeros((n, 6)), "mean_r": np.zeros(n),
        "l": np.zeros(n, np.int32), "color": np.zeros(n, np.int32),
        "n_jumps": np.zeros(n, np.int32), "status": np.zeros(n, np.int32),
        "steps_done": np.zeros(n, np.int64), "min_gap": np.zeros(n),
    }
    if want_psi:
        out["psi"] = np.zeros((n, N, 2))
    r = qt_results(*[(_dp(out[k]) if out[k].dtype == np.float64 else
                      out[k].ctypes.data_as(_I32 if out[k].dtype == np.int32 else _I64))
                     for k in ("norm", "first_r", "overlap", "survival", "mean_r", "l", "color",
                               "n_jumps", "status", "steps_done", "min_gap")],
                   _dp(out.get("psi")), None, 0, 0)
    return out, r


def to_numpy(out):
    res = {k: v.cpu().numpy() for k, v in out.items()}
    if "psi" in res:
        res["psi"] = res["psi"][..., 0] + 1j * res["psi"][..., 1]
    return res


# ---------------------------------------------------------------- context --

class Context:
    """Owns a qt_context on one HIP device."""

    def __init__(self, device=0):
        # torch carries its own HIP runtime; it has to bring the device up
        # before this library's runtime does, or torch will not see it
        try:
            import torch
            if torch.cuda.is_available():
                torch.cuda.init()
        except ImportError:
            pass
        h = _VP()
        check(lib().qt_context_create(int(device), C.byref(h)), "qt_context_create")
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            lib().qt_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_kernel_ms(self):
        ms = C.c_double()
        n = C.c_int64()
        check(lib().qt_last_kernel_ms(self.h, C.byref(ms), C.byref(n)), "qt_last_kernel_ms")
        return ms.value, n.value

    def plan_set(self, N, precision, threads_per_traj):
        """Fix the fused kernel variant for (N, precision) (qt_plan_set)."""
        check(lib().qt_plan_set(self.h, int(N), int(precision), int(threads_per_traj)),
              "qt_plan_set")

    def plan(self, N, precision, tune=False):
        w = C.c_int32()
        s = C.c_int32()
        check(lib().qt_plan(self.h, int(N), int(precision), int(bool(tune)), C.byref(w),
                            C.byref(s)), "qt_plan")
        return w.value, s.value


def eigen_basis(ctx, cfg):
    """Vacuum eigenstates 1S, 2S, 1P, 3S, 2P, 1D of the discrete Hamiltonian
    (qt_eigen_basis): (energies [6] in GeV, basis [6, N])."""
    N = int(cfg["N"])
    e = np.zeros(6)
    b = np.zeros((6, N))
    p = physics(cfg)
    check(lib().qt_eigen_basis(ctx.h, C.byref(p), e.ctypes.data_as(_D), b.ctypes.data_as(_D)),
          "qt_eigen_basis")
    return e, b


def plan_variants(N, precision):
    """Threads per trajectory of every fused kernel variant for (N, precision)
    (qt_plan_variants; host query)."""
    n = C.c_int32(0)
    buf = (C.c_int32 * 16)()
    check(lib().qt_plan_variants(int(N), int(precision), buf, 16, C.byref(n)), "qt_plan_variants")
    return [int(buf[i]) for i in range(min(n.value, 16))]


def count_steps(cfg):
    """qt_count_steps: the number of time steps a run of this config takes
    (host computation, no device)."""
    keep = []
    p = physics(cfg)
    tt = ttable(cfg, keep)
    n = C.c_int64(0)
    check(lib().qt_count_steps(C.byref(p), C.byref(tt), C.byref(n)), "qt_count_steps")
    return n.value


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def run(ctx, cfg, precision=QT_FP64, form=QT_FORM_FUSED, want_psi=False, n_traj=None,
        traj_id0=None, stream=None, out=None, jump_log_cap=0):
    """qt_run on a config dict; returns the dict of output tensors."""
    keep = []
    n = int(cfg["n_traj"] if n_traj is None else n_traj)
    if out is None:
        out, res = alloc_results(n, int(cfg["N"]), want_psi, jump_log_cap=jump_log_cap)
    else:
        res = results_struct(out)
    p = physics(cfg)
    tt = ttable(cfg, keep)
    ini = init(cfg, keep)
    b = batch(cfg, precision, form, n, traj_id0)
    check(lib().qt_run(ctx.h, C.byref(p), C.byref(tt), C.byref(ini), C.byref(b), C.byref(res),
                       _stream_handle(stream)), "qt_run")
    return out


def run_noalloc(ctx, cfg, precision=QT_FP64, want_psi=False, n_traj=None, traj_id0=None,
                stream=None, out=None):
    """qt_run_noalloc (the fused form without device allocation) on a config
    dict; `out`: result tensors of an earlier call to reuse."""
    keep = []
    n = int(cfg["n_traj"] if n_traj is None else n_traj)
    if out is None:
        out, res = alloc_results(n, int(cfg["N"]), want_psi)
    else:
        res = results_struct(out)
    p = physics(cfg)
    tt = ttable(cfg, keep)
    ini = init(cfg, keep)
    b = batch(cfg, precision, QT_FORM_FUSED, n, traj_id0)
    check(lib().qt_run_noalloc(ctx.h, C.byref(p), C.byref(tt), C.byref(ini), C.byref(b),
                               C.byref(res), _stream_handle(stream)), "qt_run_noalloc")
    return out


def run_many(ctx, cfgs, precision=QT_FP32_BULK, want_psi=False, stream=None, flat=False):
    """qt_run_many over a list of config dicts; returns one output dict each,
    or with flat=True (no wave functions) one dict holding every config's
    trajectories one after the other, in config order."""
    keep = []
    k = len(cfgs)
    P = (qt_physics * k)()
    TT = (qt_ttable * k)()
    IN = (qt_init * k)()
    B = (qt_batch * k)()
    outs = []
    if flat:
        if want_psi:
            raise ValueError("flat results hold no wave functions")
        counts = np.array([int(c["n_traj"]) for c in cfgs], dtype=np.int64)
        flat_out, _ = alloc_results(int(counts.sum()), 0, False)
        RS = results_array(flat_out, np.concatenate([[0], np.cumsum(counts)[:-1]]), keep)
    else:
        RS = (qt_results * k)()
    for i, cfg in enumerate(cfgs):
        if not flat:
            o, RS[i] = alloc_results(int(cfg["n_traj"]), int(cfg["N"]), want_psi)
            outs.append(o)
        P[i] = physics(cfg)
        TT[i] = ttable(cfg, keep)
        IN[i] = init(cfg, keep)
        B[i] = batch(cfg, precision, QT_FORM_FUSED)
    check(lib().qt_run_many(ctx.h, k, P, TT, IN, B, RS, _stream_handle(stream)), "qt_run_many")
    return flat_out if flat else outs


# -------------------------------------------------------------------- jobs --

class Job:
    """Segmented run (qt_job_*): state checkpointed in device memory every
    `segment_steps` steps; advance() replays a captured HIP graph."""

    def __init__(self, ctx, cfg, precision=QT_FP32_BULK, segment_steps=1000, n_traj=None):
        self._keep = []
        self.ctx = ctx
        self.cfg = cfg
        self.n = int(cfg["n_traj"] if n_traj is None else n_traj)
        p = physics(cfg)
        tt = ttable(cfg, self._keep)
        ini = init(cfg, self._keep)
        b = batch(cfg, precision, QT_FORM_FUSED, self.n)
        h = _VP()
        check(lib().qt_job_create(ctx.h, C.byref(p), C.byref(tt), C.byref(ini), C.byref(b),
                                  int(segment_steps), C.byref(h)), "qt_job_create")
        self.h = h

    def advance(self, steps, stream=None):
        check(lib().qt_job_advance(self.h, int(steps), _stream_handle(stream)), "qt_job_advance")

    def done(self):
        d = C.c_int32()
        check(lib().qt_job_done(self.h, C.byref(d)), "qt_job_done")
        return bool(d.value)

    def state_bytes(self):
        n = C.c_size_t()
        check(lib().qt_job_state_bytes(self.h, C.byref(n)), "qt_job_state_bytes")
        return n.value

    def save(self, dst_ptr, stream=None):
        check(lib().qt_job_save(self.h, C.c_void_p(dst_ptr), _stream_handle(stream)), "qt_job_save")

    def load(self, src_ptr, stream=None):
        check(lib().qt_job_load(self.h, C.c_void_p(src_ptr), _stream_handle(stream)), "qt_job_load")

    def results(self, want_psi=False, stream=None):
        out, res = alloc_results(self.n, int(self.cfg["N"]), want_psi)
        check(lib().qt_job_results(self.h, C.byref(res), _stream_handle(stream)), "qt_job_results")
        return out

    def close(self):
        if self.h:
            lib().qt_job_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ server --

class Server:
    """Continuous-batching server (qt_server_*)."""

    def __init__(self, ctx, precision=QT_FP32_BULK, segment_steps=500, hbm_budget_bytes=0,
                 max_occupancy=0.0):
        cfg = qt_server_cfg(int(hbm_budget_bytes), int(segment_steps), int(precision), 0,
                            float(max_occupancy))
        h = _VP()
        check(lib().qt_server_create(ctx.h, C.byref(cfg), C.byref(h)), "qt_server_create")
        self.h = h
        self.precision = precision
        self._pending = {}

    def submit(self, cfg, n_traj=None):
        keep = []
        p = physics(cfg)
        tt = ttable(cfg, keep)
        ini = init(cfg, keep)
        b = batch(cfg, self.precision, QT_FORM_FUSED, n_traj)
        rid = C.c_uint64()
        check(lib().qt_submit(self.h, C.byref(p), C.byref(tt), C.byref(ini), C.byref(b),
                              C.byref(rid)), "qt_submit")
        self._pending[rid.value] = (int(b.n_traj), int(cfg["N"]))
        return rid.value

    def poll(self, rid):
        d = C.c_int32()
        check(lib().qt_poll(self.h, C.c_uint64(rid), C.byref(d)), "qt_poll")
        return bool(d.value)

    def wait(self, rid, timeout_s=-1.0, want_psi=False):
        n, N = self._pending[rid]
        out, res = host_results(n, N, want_psi)
        check(lib().qt_wait(self.h, C.c_uint64(rid), C.byref(res), float(timeout_s)), "qt_wait")
        del self._pending[rid]
        if want_psi:
            out["psi"] = out["psi"][..., 0] + 1j * out["psi"][..., 1]
        return out

    def cancel(self, rid):
        check(lib().qt_cancel(self.h, C.c_uint64(rid)), "qt_cancel")

    def stats(self):
        st = qt_stats()
        check(lib().qt_server_stats(self.h, C.byref(st)), "qt_server_stats")
        return {k: getattr(st, k) for k, _ in qt_stats._fields_}

    def close(self):
        if self.h:
            lib().qt_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
