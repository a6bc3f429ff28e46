"""Plain FP64 CPU oracle of the Cosm sweep (ctypes wrapper over cosm_oracle.c).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
package never imports it and shares no code with it.

Phases handled here are degrees in [0, 360), the paper's unit (Sec. II-A).
Parity is pinned for: Philox (known-answer vectors), the greedy colouring
(matching invariants, hand-worked small graphs), energy and cut (Eq. (1),
Eq. (14), closed-form ground states, brute force), R99 (Tables II and VI), and
the sweep's invariants (Eqs. (4)-(6), (12)-(13), the dual window twist).  The
long-run trajectory itself has no printed reference: parity unpinned beyond
those invariants.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cosm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SCHED_GRID = 0
SCHED_CONTINUOUS = 1
SCHED_GRID16 = 2  # 16-bit grid: phases on 360 * 2^-16 degrees, steps on 360 * 2^-15
UPDATE_SCS = 0
UPDATE_FULL_GRADIENT = 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP over replicas)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int64),
                ("eu", ctypes.c_void_p), ("ev", ctypes.c_void_p), ("J", ctypes.c_void_p),
                ("h", ctypes.c_void_p), ("colour", ctypes.c_void_p), ("C", ctypes.c_int32)]


class _Params(ctypes.Structure):
    _fields_ = [("alpha0_deg", ctypes.c_double), ("dwt_ratio", ctypes.c_double),
                ("dwt_period", ctypes.c_int32), ("dwt_window_deg", ctypes.c_double),
                ("n_bisectors", ctypes.c_int32), ("sweeps", ctypes.c_int64),
                ("schedule", ctypes.c_int32), ("update", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_greedy_colouring.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, P]
        L.orc_greedy_colouring.restype = ctypes.c_int32
        L.orc_is_proper_colouring.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, P,
                                              ctypes.c_int32]
        L.orc_is_proper_colouring.restype = ctypes.c_int32
        L.orc_alpha.argtypes = [ctypes.POINTER(_Params), ctypes.c_int64]
        L.orc_alpha.restype = ctypes.c_double
        L.orc_bisector.argtypes = [ctypes.POINTER(_Params), ctypes.c_int32, ctypes.c_int32]
        L.orc_bisector.restype = ctypes.c_double
        L.orc_init_phases.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64,
                                      ctypes.c_int32, ctypes.c_int32, P]
        L.orc_theta_ref.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64]
        L.orc_theta_ref.restype = ctypes.c_double
        L.orc_theta_ref_sched.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64,
                                          ctypes.c_int32]
        L.orc_theta_ref_sched.restype = ctypes.c_double
        L.orc_twist_direction.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64]
        L.orc_twist_direction.restype = ctypes.c_int32
        L.orc_sweeps.argtypes = [ctypes.POINTER(_Problem), ctypes.POINTER(_Params),
                                 ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32,
                                 ctypes.c_int64, ctypes.c_int64, P, P, ctypes.c_int64,
                                 ctypes.c_int32]
        L.orc_sweeps.restype = ctypes.c_int32
        L.orc_energy.argtypes = [ctypes.POINTER(_Problem), ctypes.c_int32, P, P, P]
        L.orc_coupling_v.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_coupling_v.restype = ctypes.c_double
        L.orc_relaxed_objective.argtypes = [ctypes.POINTER(_Problem), ctypes.c_int32, P, P]
        L.orc_readout.argtypes = [ctypes.POINTER(_Problem), ctypes.POINTER(_Params),
                                  ctypes.c_int32, P, P, P, P, P]
        L.orc_readout_optimal.argtypes = [ctypes.POINTER(_Problem), ctypes.c_int32, P, P, P, P, P]
        L.orc_readout_optimal.restype = ctypes.c_int32
        L.orc_brute_force_ground_state.argtypes = [ctypes.POINTER(_Problem), P, P]
        L.orc_brute_force_ground_state.restype = ctypes.c_int32
        L.orc_r99.argtypes = [ctypes.c_double]
        L.orc_r99.restype = ctypes.c_double
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def greedy_colouring(n, eu, ev):
    eu = np.ascontiguousarray(eu, dtype=np.int32)
    ev = np.ascontiguousarray(ev, dtype=np.int32)
    colour = np.zeros(len(eu), dtype=np.int32)
    C = lib().orc_greedy_colouring(n, len(eu), _ptr(eu), _ptr(ev), _ptr(colour))
    if C < 0:
        raise ValueError("invalid edge list")
    return colour, C


def is_proper_colouring(n, eu, ev, colour, C):
    eu = np.ascontiguousarray(eu, dtype=np.int32)
    ev = np.ascontiguousarray(ev, dtype=np.int32)
    colour = np.ascontiguousarray(colour, dtype=np.int32)
    return bool(lib().orc_is_proper_colouring(n, len(eu), _ptr(eu), _ptr(ev), _ptr(colour), C))


class Problem:
    """An instance: n spins, edges (eu[k], ev[k]) with Ising coupling J[k], optional
    bias h, and a colouring (class of each edge, classes applied in index order)."""

    def __init__(self, n, eu, ev, J, colour=None, C=None, h=None):
        self.n = int(n)
        self.eu = np.ascontiguousarray(eu, dtype=np.int32)
        self.ev = np.ascontiguousarray(ev, dtype=np.int32)
        self.J = np.ascontiguousarray(J, dtype=np.int32)
        self.h = None if h is None else np.ascontiguousarray(h, dtype=np.int32)
        if colour is None:
            colour, C = greedy_colouring(self.n, self.eu, self.ev)
        self.colour = np.ascontiguousarray(colour, dtype=np.int32)
        self.C = int(C if C is not None else (int(self.colour.max()) + 1 if len(self.colour) else 0))
        self._s = _Problem(self.n, len(self.eu), _ptr(self.eu), _ptr(self.ev), _ptr(self.J),
                           _ptr(self.h), _ptr(self.colour), self.C)

    @property
    def m(self):
        return len(self.eu)

    def struct(self):
        return ctypes.byref(self._s)


class Params:
    def __init__(self, alpha0_deg=14.0, dwt_ratio=0.5, dwt_period=3, dwt_window_deg=90.0,
                 n_bisectors=100, sweeps=1000, schedule=SCHED_GRID, update=UPDATE_SCS):
        self.alpha0_deg = float(alpha0_deg)
        self.dwt_ratio = float(dwt_ratio)
        self.dwt_period = int(dwt_period)
        self.dwt_window_deg = float(dwt_window_deg)
        self.n_bisectors = int(n_bisectors)
        self.sweeps = int(sweeps)
        self.schedule = int(schedule)
        self.update = int(update)

    def struct(self):
        return ctypes.byref(_Params(self.alpha0_deg, self.dwt_ratio, self.dwt_period,
                                    self.dwt_window_deg, self.n_bisectors, self.sweeps,
                                    self.schedule, self.update))


def alpha(params: Params, t: int) -> float:
    return lib().orc_alpha(params.struct(), t)


def bisector(params: Params, idx: int) -> float:
    return lib().orc_bisector(params.struct(), params.schedule, idx)


def theta_ref(seed: int, t: int, rid: int, schedule=SCHED_GRID) -> float:
    return lib().orc_theta_ref_sched(seed, t, rid, schedule)


def twist_direction(seed: int, t: int, rid: int) -> int:
    """+1 / -1: the twist sense drawn per event when bias fields are present."""
    return lib().orc_twist_direction(seed, t, rid)


def init_phases(n, seed, rid0, R, schedule=SCHED_GRID):
    x = np.zeros((R, n), dtype=np.float64)
    lib().orc_init_phases(n, seed, rid0, R, schedule, _ptr(x))
    return x


def sweeps(problem: Problem, params: Params, seed, rid0, x, t_from, n_sweeps,
           diag_sweeps=0, n_threads=0):
    """Advance x ([R][n] degrees, modified in place) by n_sweeps sweeps starting
    after sweep t_from.  Returns per-replica near-tie margins (degrees) over the
    first diag_sweeps sweeps when diag_sweeps > 0, else None."""
    assert x.dtype == np.float64 and x.flags.c_contiguous and x.shape[1] == problem.n
    R = x.shape[0]
    margin = np.zeros(R, dtype=np.float64) if diag_sweeps > 0 else None
    rc = lib().orc_sweeps(problem.struct(), params.struct(), seed, rid0, R, t_from, n_sweeps,
                          _ptr(x), _ptr(margin), diag_sweeps, n_threads)
    if rc != 0:
        raise ValueError("orc_sweeps rejected its arguments")
    return margin


def energy(problem: Problem, spins):
    s = np.ascontiguousarray(spins, dtype=np.int8)
    if s.ndim == 1:
        s = s[None, :]
    R = s.shape[0]
    H = np.zeros(R, dtype=np.int64)
    cut = np.zeros(R, dtype=np.int64)
    lib().orc_energy(problem.struct(), R, _ptr(s), _ptr(H), _ptr(cut))
    return H, cut


def coupling_v(xi_deg: float, xj_deg: float) -> float:
    """Relaxed coupling v of Eq. (2), phases in degrees."""
    return float(lib().orc_coupling_v(float(xi_deg), float(xj_deg)))


def relaxed_objective(problem: Problem, x):
    """Relaxed objective f(x) of Eq. (7) for x ([R][n] or [n], degrees)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[None, :]
    f = np.zeros(x.shape[0], dtype=np.float64)
    lib().orc_relaxed_objective(problem.struct(), x.shape[0], _ptr(x), _ptr(f))
    return f


def readout(problem: Problem, params: Params, x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    R = x.shape[0]
    spins = np.zeros((R, problem.n), dtype=np.int8)
    H = np.zeros(R, dtype=np.int64)
    cut = np.zeros(R, dtype=np.int64)
    bp = np.zeros(R, dtype=np.int32)
    lib().orc_readout(problem.struct(), params.struct(), R, _ptr(x), _ptr(spins), _ptr(H),
                      _ptr(cut), _ptr(bp))
    return spins, H, cut, bp


def readout_optimal(problem: Problem, x):
    """Optimal-bisector binarization of x ([R][n], degrees).
    Returns (spins, H, cut, beta_deg)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    R = x.shape[0]
    spins = np.zeros((R, problem.n), dtype=np.int8)
    H = np.zeros(R, dtype=np.int64)
    cut = np.zeros(R, dtype=np.int64)
    beta = np.zeros(R, dtype=np.float64)
    if lib().orc_readout_optimal(problem.struct(), R, _ptr(x), _ptr(spins), _ptr(H), _ptr(cut),
                                 _ptr(beta)) != 0:
        raise ValueError("the optimal bisector needs h = 0")
    return spins, H, cut, beta


def brute_force_ground_state(problem: Problem):
    s = np.zeros(problem.n, dtype=np.int8)
    H = np.zeros(1, dtype=np.int64)
    if lib().orc_brute_force_ground_state(problem.struct(), _ptr(s), _ptr(H)) != 0:
        raise ValueError("too many spins for exhaustive search")
    return s, int(H[0])


def r99(ps: float) -> float:
    return lib().orc_r99(ps)


def solve(problem: Problem, params: Params, seed, rid0, R, n_threads=0):
    """A whole trial batch, Algorithm 1: init, S sweeps, readout.
    Returns (x, spins, H, cut)."""
    x = init_phases(problem.n, seed, rid0, R, params.schedule)
    sweeps(problem, params, seed, rid0, x, 0, params.sweeps, n_threads=n_threads)
    spins, H, cut, _ = readout(problem, params, x)
    return x, spins, H, cut
