"""CPU FP64 oracle for the QTraj quantum-trajectory solver (arXiv:2107.06147).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The GPU library and
its Python binding never import it, and it never imports them.

`build()` compiles `qtraj_oracle.c` with gcc (OpenMP) into `liboracle.so` next
to this file.  `run()` marshals numpy arrays into the C structs of
`qtraj_oracle.h` and returns a dict of numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qtraj_oracle.c")
# QTO_LIB: another build of the oracle (the mutation tests load deliberately
# broken copies through it in child processes)
_LIB_PATH = os.environ.get("QTO_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

SINGLET, OCTET = 0, 1
INIT_COULOMB, INIT_GAUSSIAN, INIT_ARRAY, INIT_EIGEN = 0, 1, 2, 3
BASIS_COULOMB, BASIS_EIGEN = 0, 1
STATUS_OK, STATUS_RMAX, STATUS_MAXJUMPS, STATUS_NOJUMP = 0, 1, 2, 4
POTENTIAL_MUNICH, POTENTIAL_KSU = 0, 1
FLAG_KINETIC_OFF = 1
BASIS = ("1S", "2S", "1P", "3S", "2P", "1D")


def build(force: bool = True) -> str:
    """Compile the oracle into liboracle.so (gcc -O2 -fopenmp)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Physics(C.Structure):
    _fields_ = [("N", C.c_int32), ("L", C.c_double), ("dt", C.c_double),
                ("mass", C.c_double), ("alpha_s", C.c_double),
                ("kappa_hat", C.c_double), ("gamma_hat", C.c_double),
                ("deriv_type", C.c_int32), ("do_jumps", C.c_int32),
                ("max_jumps", C.c_int32), ("r_max", C.c_double),
                ("flags", C.c_int32), ("potential", C.c_int32), ("md_factor", C.c_double),
                ("basis", C.POINTER(C.c_double))]


class _TTable(C.Structure):
    _fields_ = [("tau", C.POINTER(C.c_double)), ("T", C.POINTER(C.c_double)),
                ("n", C.c_int32), ("tau_start", C.c_double),
                ("T_final", C.c_double), ("max_steps", C.c_int64),
                ("vacuum_steps", C.c_int64)]


class _Init(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32), ("l", C.c_int32),
                ("color", C.c_int32), ("width", C.c_double),
                ("u_re", C.POINTER(C.c_double)), ("u_im", C.POINTER(C.c_double))]


class _Batch(C.Structure):
    _fields_ = [("n_traj", C.c_int64), ("seed", C.c_uint64), ("traj_id0", C.c_uint64),
                ("traj_id_stride", C.c_uint64), ("no_jump_shortcut", C.c_int32)]


_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)
_I64 = C.POINTER(C.c_int64)


class _Results(C.Structure):
    _fields_ = [("norm", _D), ("first_r", _D), ("overlap", _D), ("survival", _D),
                ("mean_r", _D), ("l", _I32), ("color", _I32), ("n_jumps", _I32),
                ("status", _I32), ("steps_done", _I64), ("min_gap", _D),
                ("psi", _D), ("norm_trace", _D), ("jump_log_cap", C.c_int32),
                ("jump_log", _D)]


def lib():
    """Load liboracle.so, building it first only if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = C.CDLL(_LIB_PATH)
        L.qto_run.argtypes = [C.POINTER(_Physics), C.POINTER(_TTable), C.POINTER(_Init),
                              C.POINTER(_Batch), C.POINTER(_Results), C.c_int]
        L.qto_run.restype = C.c_int
        L.qto_num_steps.argtypes = [C.POINTER(_Physics), C.POINTER(_TTable)]
        L.qto_num_steps.restype = C.c_int64
        L.qto_philox4x64_10.argtypes = [C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                        C.POINTER(C.c_uint64)]
        L.qto_philox4x64_10.restype = None
        L.qto_uniform.argtypes = [C.c_uint64]
        L.qto_uniform.restype = C.c_double
        L.qto_dst1.argtypes = [C.c_int32, _D, _D, _D, _D]
        L.qto_dst1.restype = None
        L.qto_jump_rule.argtypes = [C.c_uint64, C.c_uint64, C.c_int64, C.c_int32, C.c_int32,
                                    _I32, _I32]
        L.qto_jump_rule.restype = None
        L.qto_basis_state.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double,
                                      C.c_int32, C.c_int32, _D]
        L.qto_basis_state.restype = C.c_int
        L.qto_temperature.argtypes = [C.POINTER(_TTable), C.c_double]
        L.qto_temperature.restype = C.c_double
        L.qto_kappa_hat.argtypes = [C.c_double, C.c_double]
        L.qto_kappa_hat.restype = C.c_double
        L.qto_ksu_phi.argtypes = [C.c_double]
        L.qto_ksu_phi.restype = C.c_double
        L.qto_potential.argtypes = [C.POINTER(_Physics), C.c_double, C.c_int32, C.c_int32,
                                    C.c_double, _D, _D]
        L.qto_potential.restype = None
        L.qto_kinetic_energy.argtypes = [C.POINTER(_Physics), C.c_int32]
        L.qto_kinetic_energy.restype = C.c_double
        _lib = L
    return _lib


def _dptr(a):
    return None if a is None else a.ctypes.data_as(_D)


def _physics(cfg, basis=None):
    return _Physics(int(cfg["N"]), float(cfg["L"]), float(cfg["dt"]), float(cfg["mass"]),
                    float(cfg["alpha_s"]), float(cfg["kappa_hat"]), float(cfg["gamma_hat"]),
                    int(cfg.get("deriv_type", 0)), int(cfg.get("do_jumps", 1)),
                    int(cfg.get("max_jumps", -1)), float(cfg.get("r_max", 1.0)),
                    int(cfg.get("flags", 0)), int(cfg.get("potential", 0)),
                    float(cfg.get("md_factor", 1.0)), _dptr(basis))


def _ttable(cfg, keep):
    tau = np.ascontiguousarray(cfg["tau"], dtype=np.float64)
    T = np.ascontiguousarray(cfg["T"], dtype=np.float64)
    keep += [tau, T]
    return _TTable(_dptr(tau), _dptr(T), len(tau), float(cfg["tau_start"]),
                   float(cfg.get("T_final", 0.0)), int(cfg.get("max_steps", 2**62)),
                   int(cfg.get("vacuum_steps", 0)))


def _init(cfg, keep):
    kind = int(cfg.get("init_kind", INIT_COULOMB))
    u_re = u_im = None
    if kind == INIT_ARRAY:
        u = np.asarray(cfg["u0"])
        u_re = np.ascontiguousarray(u.real, dtype=np.float64)
        u_im = np.ascontiguousarray(u.imag, dtype=np.float64)
        keep += [u_re, u_im]
    return _Init(kind, int(cfg.get("init_n", 1)), int(cfg.get("init_l", 0)),
                 int(cfg.get("init_color", SINGLET)), float(cfg.get("init_width", 0.0)),
                 _dptr(u_re), _dptr(u_im))


def num_steps(cfg) -> int:
    keep = []
    p = _physics(cfg)
    tt = _ttable(cfg, keep)
    return int(lib().qto_num_steps(C.byref(p), C.byref(tt)))


def run(cfg, n_traj=None, traj_id0=None, want_psi=False, want_trace=False,
        jump_log_cap=0, n_threads=0):
    """Run the oracle on a config dict (see paper_2107_06147_amd.workloads)."""
    keep = []
    n = int(cfg["n_traj"] if n_traj is None else n_traj)
    t0 = int(cfg.get("traj_id0", 0) if traj_id0 is None else traj_id0)
    basis = None
    if int(cfg.get("basis", BASIS_COULOMB)) == BASIS_EIGEN or \
            int(cfg.get("init_kind", INIT_COULOMB)) == INIT_EIGEN:
        _, eig = eigen_basis(cfg)
        if int(cfg.get("basis", BASIS_COULOMB)) == BASIS_EIGEN:
            basis = np.ascontiguousarray(eig)
            keep.append(basis)
        if int(cfg.get("init_kind", INIT_COULOMB)) == INIT_EIGEN:
            # initType 100: the eigenstate (n, l) as an array initial state
            slot = [(1, 0), (2, 0), (2, 1), (3, 0), (3, 1), (3, 2)].index(
                (int(cfg.get("init_n", 1)), int(cfg.get("init_l", 0))))
            cfg = dict(cfg, init_kind=INIT_ARRAY, u0=eig[slot].astype(complex))
    p = _physics(cfg, basis)
    tt = _ttable(cfg, keep)
    ini = _init(cfg, keep)
    b = _Batch(n, int(cfg.get("seed", 1)), t0, int(cfg.get("traj_id_stride", 1)),
               int(cfg.get("no_jump_shortcut", 0)))
    n_steps = int(lib().qto_num_steps(C.byref(p), C.byref(tt)))
    N = int(cfg["N"])
    out = {
        "norm": np.zeros(n), "first_r": np.zeros(n), "overlap": np.zeros((n, 6)),
        "survival": np.zeros((n, 6)), "mean_r": np.zeros(n),
        "l": np.zeros(n, np.int32), "color": np.zeros(n, np.int32),
        "n_jumps": np.zeros(n, np.int32), "status": np.zeros(n, np.int32),
        "steps_done": np.zeros(n, np.int64), "min_gap": np.zeros(n),
    }
    if want_psi:
        out["psi"] = np.zeros((n, N, 2))
    if want_trace:
        out["norm_trace"] = np.zeros((n, n_steps))
    if jump_log_cap:
        out["jump_log"] = np.zeros((n, jump_log_cap, 5))
    res = _Results(
        _dptr(out["norm"]), _dptr(out["first_r"]), _dptr(out["overlap"]),
        _dptr(out["survival"]), _dptr(out["mean_r"]),
        out["l"].ctypes.data_as(_I32), out["color"].ctypes.data_as(_I32),
        out["n_jumps"].ctypes.data_as(_I32), out["status"].ctypes.data_as(_I32),
        out["steps_done"].ctypes.data_as(_I64), _dptr(out["min_gap"]),
        _dptr(out.get("psi")), _dptr(out.get("norm_trace")), int(jump_log_cap),
        _dptr(out.get("jump_log")))
    rc = lib().qto_run(C.byref(p), C.byref(tt), C.byref(ini), C.byref(b), C.byref(res),
                       int(n_threads))
    if rc != 0:
        raise ValueError("oracle rejected the input (code %d)" % rc)
    if want_psi:
        out["psi"] = out["psi"][..., 0] + 1j * out["psi"][..., 1]
    out["n_steps"] = n_steps
    out["init_l"] = int(cfg.get("init_l", 0))
    out["init_color"] = int(cfg.get("init_color", SINGLET))
    return out


def philox(ctr, key):
    c = (C.c_uint64 * 4)(*[int(x) & (2**64 - 1) for x in ctr])
    k = (C.c_uint64 * 2)(*[int(x) & (2**64 - 1) for x in key])
    o = (C.c_uint64 * 4)()
    lib().qto_philox4x64_10(c, k, o)
    return [int(x) for x in o]


def uniform(word):
    return float(lib().qto_uniform(C.c_uint64(int(word))))


def dst1(x):
    x = np.asarray(x, dtype=np.complex128)
    N = len(x)
    re = np.ascontiguousarray(x.real)
    im = np.ascontiguousarray(x.imag)
    ore = np.zeros(N)
    oim = np.zeros(N)
    lib().qto_dst1(N, _dptr(re), _dptr(im), _dptr(ore), _dptr(oim))
    return ore + 1j * oim


def jump_rule(seed, traj_id, event, l, c):
    ln = C.c_int32()
    cn = C.c_int32()
    lib().qto_jump_rule(seed, traj_id, event, l, c, C.byref(ln), C.byref(cn))
    return ln.value, cn.value


def basis_state(N, L, mass, alpha_s, n, l):
    u = np.zeros(N)
    rc = lib().qto_basis_state(N, L, mass, alpha_s, n, l, _dptr(u))
    if rc != 0:
        raise ValueError("no such basis state")
    return u


def temperature(cfg, t):
    keep = []
    tt = _ttable(cfg, keep)
    return float(lib().qto_temperature(C.byref(tt), float(t)))


def kappa_hat(kappa_hat_param, T):
    """kappa_hat at temperature T (a constant, or one of the fits -1/-2/-3)."""
    return float(lib().qto_kappa_hat(float(kappa_hat_param), float(T)))


def ksu_phi(a):
    """phi(a) of the imaginary part of the isotropic KSU potential."""
    return float(lib().qto_ksu_phi(float(a)))


def potential(cfg, r, l, color=SINGLET, T=0.0):
    """(V_R, V_I) of the configured potential at r."""
    p = _physics(cfg)
    vr, vi = C.c_double(), C.c_double()
    lib().qto_potential(C.byref(p), float(r), int(l), int(color), float(T), C.byref(vr), C.byref(vi))
    return vr.value, vi.value


_EIGEN_CACHE = {}


def eigen_basis(cfg):
    """Vacuum eigenstates 1S, 2S, 1P, 3S, 2P, 1D (Sec. "Using the built-in
    eigensolvers"): the eigenvectors of the discrete Hamiltonian that the
    evolution uses, at T = 0 for a singlet, H = T_kin + V with
      T_kin = (2/N) S diag(E_k) S,  S_mk = sin(pi m k / N),  m, k = 1..N-1,
    (E_k the kinetic energy of sine mode k, Sec. "Derivative types") and V the
    potential plus the centrifugal term at r_m = m dr.  H is built as a dense
    FP64 matrix and diagonalised (numpy.linalg.eigh); state n_r of angular
    momentum l is the (n_r + 1)-th lowest.  Each state is normalised to
    dr sum u_m^2 = 1 with u_1 > 0.  Returns (energies [6], basis [6, N])."""
    key = (int(cfg["N"]), float(cfg["L"]), float(cfg["mass"]), float(cfg["alpha_s"]),
           int(cfg.get("deriv_type", 0)), int(cfg.get("potential", 0)))
    if key in _EIGEN_CACHE:
        e, b = _EIGEN_CACHE[key]
        return e.copy(), b.copy()
    N = int(cfg["N"])
    dr = float(cfg["L"]) / N
    p = _physics(cfg)
    m = np.arange(1, N)
    S = np.sin(np.pi * np.outer(m, m) / N)
    E = np.array([lib().qto_kinetic_energy(C.byref(p), int(k)) for k in m])
    Tk = (2.0 / N) * ((S * E) @ S)
    energies = np.zeros(6)
    basis = np.zeros((6, N))
    for l, slots in ((0, (0, 1, 3)), (1, (2, 4)), (2, (5,))):
        V = np.array([potential(cfg, j * dr, l)[0] for j in m])
        w, v = np.linalg.eigh(Tk + np.diag(V))
        for nr, b in enumerate(slots):
            u = v[:, nr] / np.sqrt(dr * np.sum(v[:, nr] ** 2))
            if u[0] < 0:
                u = -u
            energies[b] = w[nr]
            basis[b, 1:] = u
    _EIGEN_CACHE[key] = (energies.copy(), basis.copy())
    return energies, basis
