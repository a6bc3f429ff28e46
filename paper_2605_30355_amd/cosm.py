"""ctypes binding of libcosm (include/cosm.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libcosm.so")

COSM_OK = 0
STATUS_NAMES = {0: "COSM_OK", -1: "COSM_EINVAL", -2: "COSM_EDUP", -3: "COSM_ECOLOR",
                -4: "COSM_ERANGE", -5: "COSM_ENOMEM", -6: "COSM_EDEVICE", -7: "COSM_ESTATE"}
COLOR_GREEDY, COLOR_MISRA_GRIES, COLOR_TORUS, COLOR_BALANCED, COLOR_MINIMUM = 0, 1, 2, 3, 4
STORE_FP32, STORE_FP16, STORE_BF16, STORE_FIX16, STORE_FIX32, STORE_FP16_PK = 0, 1, 2, 3, 4, 5
ORDER_LARGEST_LAST = 0x100  # OR into a colouring method: the largest class goes last
RES_AUTO, RES_LDS, RES_HBM, RES_PLAIN = 0, 1, 2, 3
SCHED_GRID, SCHED_CONTINUOUS = 0, 1
UPDATE_SCS, UPDATE_FULL_GRADIENT = 0, 1
READOUT_BISECTORS, READOUT_OPTIMAL = 0, 1
UNIT_TURNS, UNIT_DEGREES, UNIT_RADIANS = 0, 1, 2
LDS_FORM_AUTO, LDS_FORM_PAIR, LDS_FORM_REGISTER, LDS_FORM_REGISTER_STREAM = 0, 1, 2, 3

# Every function declared in include/cosm.h.
ABI_FUNCTIONS = (
    "cosm_default_params", "cosm_build_partitions", "cosm_workspace_bytes", "cosm_init",
    "cosm_init_static",
    "cosm_destroy", "cosm_reset", "cosm_sweep", "cosm_energy", "cosm_solve_to_target",
    "cosm_get_phases", "cosm_set_phases", "cosm_get_info", "cosm_set_timing",
    "cosm_last_error", "cosm_version", "cosm_lds_probe", "cosm_qubo_to_ising",
    "cosm_batch_create", "cosm_batch_destroy", "cosm_batch_add_graph", "cosm_batch_set_seed",
    "cosm_batch_run", "cosm_batch_wait", "cosm_batch_poll", "cosm_batch_results",
    "cosm_batch_graph_shape",
)


class CosmError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")


class _CParams(ctypes.Structure):
    _fields_ = [("alpha0_deg", ctypes.c_double), ("dwt_ratio", ctypes.c_double),
                ("dwt_period", ctypes.c_int32), ("dwt_window_deg", ctypes.c_double),
                ("n_bisectors", ctypes.c_int32), ("sweeps_per_trial", ctypes.c_int64),
                ("schedule", ctypes.c_int32), ("storage", ctypes.c_int32),
                ("residency", ctypes.c_int32), ("replicas_per_wg", ctypes.c_int32),
                ("threads_per_wg", ctypes.c_int32), ("update", ctypes.c_int32),
                ("readout", ctypes.c_int32), ("lds_form", ctypes.c_int32)]


class _CTTS(ctypes.Structure):
    _fields_ = [("trials", ctypes.c_int64), ("successes", ctypes.c_int64),
                ("ps", ctypes.c_double), ("ps_lo", ctypes.c_double), ("ps_hi", ctypes.c_double),
                ("r99", ctypes.c_double), ("t_trial_s", ctypes.c_double),
                ("ttt_s", ctypes.c_double), ("stt_sweeps", ctypes.c_double),
                ("best_H", ctypes.c_int64), ("best_cut", ctypes.c_int64)]


class _CInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("num_colours", ctypes.c_int32),
                ("replicas", ctypes.c_int32), ("m", ctypes.c_int64),
                ("sweeps_done", ctypes.c_int64), ("residency", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("replicas_per_wg", ctypes.c_int32),
                ("threads_per_wg", ctypes.c_int32), ("workgroups", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int32), ("max_class_edges", ctypes.c_int32),
                ("sweep_launches", ctypes.c_int64), ("sweep_kernel_ms", ctypes.c_double),
                ("lds_form", ctypes.c_int32), ("register_rows", ctypes.c_int32),
                ("twist_fused", ctypes.c_int32), ("register_vertices", ctypes.c_int32),
                ("register_edges", ctypes.c_int64), ("streamed", ctypes.c_int32),
                ("lazy_wrap", ctypes.c_int32)]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Load libcosm.so (torch is imported first so that one HIP runtime serves both)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise CosmError(-6, f"{_LIB_PATH} is not built: run `python {os.path.join(_HERE, 'build.py')}`")
    import torch  # noqa: F401  (loads the HIP runtime torch was built with)
    L = ctypes.CDLL(_LIB_PATH)
    P, I32, I64, U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    PS = ctypes.POINTER(_CParams)
    sig = {
        "cosm_default_params": (None, [PS]),
        "cosm_build_partitions": (I32, [I32, I64, P, P, I32, P, P, P]),
        "cosm_workspace_bytes": (I32, [I32, I64, I32, I32, PS, ctypes.POINTER(ctypes.c_size_t)]),
        "cosm_init": (I32, [ctypes.POINTER(P), I32, I64, P, P, P, P, P, I32, PS, U64, I32, P, P,
                            ctypes.c_size_t]),
        "cosm_init_static": (I32, [ctypes.POINTER(P), I32, I64, P, P, P, P, P, I32, PS, U64, I32,
                                   P]),
        "cosm_destroy": (I32, [P]),
        "cosm_reset": (I32, [P, U64, I64]),
        "cosm_sweep": (I32, [P, I64]),
        "cosm_energy": (I32, [P, P, P, P, P]),
        "cosm_solve_to_target": (I32, [P, I64, I64, I32, ctypes.POINTER(_CTTS), P]),
        "cosm_get_phases": (I32, [P, I32, P]),
        "cosm_set_phases": (I32, [P, I32, P, I64]),
        "cosm_get_info": (I32, [P, ctypes.POINTER(_CInfo)]),
        "cosm_set_timing": (I32, [P, I32]),
        "cosm_last_error": (ctypes.c_char_p, []),
        "cosm_batch_create": (I32, [ctypes.POINTER(P), I32, I32, I32, I32, P]),
        "cosm_batch_destroy": (I32, [P]),
        "cosm_batch_add_graph": (I32, [P, I32, I64, P, P, P, P, I32, PS, U64, I32,
                                       ctypes.POINTER(I32)]),
        "cosm_batch_set_seed": (I32, [P, I32, U64, I64]),
        "cosm_batch_run": (I32, [P, P, I32]),
        "cosm_batch_wait": (I32, [P, ctypes.POINTER(ctypes.c_double)]),
        "cosm_batch_poll": (I32, [P, ctypes.POINTER(ctypes.c_int32)]),
        "cosm_batch_results": (I32, [P, I32, P, P, P]),
        "cosm_batch_graph_shape": (I32, [P, I32, ctypes.POINTER(I32), ctypes.POINTER(I32),
                                         ctypes.POINTER(I32), ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(I32)]),
        "cosm_version": (ctypes.c_char_p, []),
        "cosm_lds_probe": (I32, [I32, I32, P, ctypes.POINTER(ctypes.c_double)]),
        "cosm_qubo_to_ising": (I32, [I32, I64, P, P, P, P, P, P, ctypes.POINTER(ctypes.c_int64), P,
                                     ctypes.POINTER(ctypes.c_int64)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def exported_symbols():
    """Names from include/cosm.h that the loaded library exports."""
    L = load_library()
    return [name for name in ABI_FUNCTIONS if hasattr(L, name)]


def version() -> str:
    return load_library().cosm_version().decode()


def qubo_to_ising(n: int, qi, qj, qv):
    """cosm_qubo_to_ising: returns (eu, ev, J, h, offset) with 4 E(x) = H(s) + offset."""
    qi = np.ascontiguousarray(qi, dtype=np.int32)
    qj = np.ascontiguousarray(qj, dtype=np.int32)
    qv = np.ascontiguousarray(qv, dtype=np.int32)
    nnz = len(qi)
    eu = np.zeros(max(nnz, 1), np.int32)
    ev = np.zeros(max(nnz, 1), np.int32)
    J = np.zeros(max(nnz, 1), np.int32)
    h = np.zeros(n, np.int32)
    m = ctypes.c_int64(0)
    off = ctypes.c_int64(0)
    _check(load_library().cosm_qubo_to_ising(int(n), int(nnz), _ptr(qi), _ptr(qj), _ptr(qv),
                                             _ptr(eu), _ptr(ev), _ptr(J), ctypes.byref(m),
                                             _ptr(h), ctypes.byref(off)))
    k = m.value
    return eu[:k].copy(), ev[:k].copy(), J[:k].copy(), h, off.value


def lds_probe(row_words: int = 2, blocks_per_cu: int = 2) -> float:
    """LDS ceiling of the device for the sweep's read/update/write mix, GB/s
    (cosm_lds_probe), on torch's current stream."""
    import torch
    out = ctypes.c_double(0.0)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _check(load_library().cosm_lds_probe(int(row_words), int(blocks_per_cu), stream,
                                         ctypes.byref(out)))
    return out.value


def _check(status: int):
    if status != COSM_OK:
        msg = load_library().cosm_last_error().decode(errors="replace")
        raise CosmError(status, msg)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


@dataclass
class Params:
    alpha0_deg: float = 14.0
    dwt_ratio: float = 0.5
    dwt_period: int = 3
    dwt_window_deg: float = 90.0
    n_bisectors: int = 100
    sweeps_per_trial: int = 1000
    schedule: int = SCHED_GRID
    storage: int = STORE_FP32
    residency: int = RES_AUTO
    replicas_per_wg: int = 0
    threads_per_wg: int = 0
    update: int = UPDATE_SCS
    readout: int = READOUT_BISECTORS
    lds_form: int = LDS_FORM_AUTO

    def _c(self) -> _CParams:
        return _CParams(self.alpha0_deg, self.dwt_ratio, self.dwt_period, self.dwt_window_deg,
                        self.n_bisectors, self.sweeps_per_trial, self.schedule, self.storage,
                        self.residency, self.replicas_per_wg, self.threads_per_wg, self.update,
                        self.readout, self.lds_form)


def default_params() -> Params:
    c = _CParams()
    load_library().cosm_default_params(ctypes.byref(c))
    return Params(*(getattr(c, f) for f, _ in _CParams._fields_))


def build_partitions(n, eu, ev, method=COLOR_GREEDY, torus_sides=None):
    """Proper edge colouring (host only).  Returns (colour[m] int32, C)."""
    L = load_library()
    eu, ev = _i32(eu), _i32(ev)
    colour = np.zeros(len(eu), dtype=np.int32)
    C = ctypes.c_int32(0)
    args = None if torus_sides is None else _i32(torus_sides)
    _check(L.cosm_build_partitions(int(n), len(eu), _ptr(eu), _ptr(ev), int(method), _ptr(args),
                                   _ptr(colour), ctypes.byref(C)))
    return colour, int(C.value)


@dataclass
class TTSResult:
    trials: int
    successes: int
    ps: float
    ps_lo: float
    ps_hi: float
    r99: float
    t_trial_s: float
    ttt_s: float
    stt_sweeps: float
    best_H: int
    best_cut: int


class State:
    """A cosm_state: one instance, R replicas, phases resident on the GPU.

    Device memory comes from a torch uint8 tensor (the workspace) and every
    kernel runs on torch's current HIP stream of the current device."""

    def __init__(self, n, eu, ev, J, colour, num_colours, params: Params | None = None, seed=0,
                 replicas=1, h=None, torch_workspace=True, static_scratch=False):
        import torch
        L = load_library()
        if not torch.cuda.is_available():
            raise CosmError(-6, "no HIP device is visible")
        self.params = params if params is not None else Params()
        self.n = int(n)
        self.R = int(replicas)
        self._eu, self._ev, self._J = _i32(eu), _i32(ev), _i32(J)
        self._colour = _i32(colour)
        self._h = None if h is None else _i32(h)
        self.m = len(self._eu)
        cp = self.params._c()
        self._stream = torch.cuda.current_stream()
        self._ws = None
        ws_ptr, ws_bytes = None, 0
        if static_scratch:  # cosm_init_static: the library's fixed per-device array
            handle = ctypes.c_void_p()
            _check(L.cosm_init_static(ctypes.byref(handle), self.n, self.m, _ptr(self._eu),
                                      _ptr(self._ev), _ptr(self._J), _ptr(self._h),
                                      _ptr(self._colour), int(num_colours), ctypes.byref(cp),
                                      int(seed) & ((1 << 64) - 1), self.R,
                                      ctypes.c_void_p(self._stream.cuda_stream)))
            self._h_state = handle
            return
        if torch_workspace:
            nbytes = ctypes.c_size_t(0)
            _check(L.cosm_workspace_bytes(self.n, self.m, int(num_colours), self.R,
                                          ctypes.byref(cp), ctypes.byref(nbytes)))
            self._ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device="cuda")
            ws_ptr, ws_bytes = ctypes.c_void_p(self._ws.data_ptr()), int(nbytes.value)
        handle = ctypes.c_void_p()
        _check(L.cosm_init(ctypes.byref(handle), self.n, self.m, _ptr(self._eu), _ptr(self._ev),
                           _ptr(self._J), _ptr(self._h), _ptr(self._colour), int(num_colours),
                           ctypes.byref(cp), int(seed) & ((1 << 64) - 1), self.R,
                           ctypes.c_void_p(self._stream.cuda_stream), ws_ptr, ws_bytes))
        self._h_state = handle

    # -- lifetime ----------------------------------------------------------------
    def close(self):
        if getattr(self, "_h_state", None):
            load_library().cosm_destroy(self._h_state)
            self._h_state = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- the method ----------------------------------------------------------------
    def sweep(self, n_sweeps: int):
        _check(load_library().cosm_sweep(self._h_state, int(n_sweeps)))

    def reset(self, seed: int, replica_offset: int = 0):
        _check(load_library().cosm_reset(self._h_state, int(seed) & ((1 << 64) - 1),
                                         int(replica_offset)))

    def energy(self, spins=None, return_spins=True):
        """Readout (spins=None) or energies of given spins [R][n].
        Returns (H[R], cut[R], spins[R][n] or None)."""
        H = np.zeros(self.R, dtype=np.int64)
        cut = np.zeros(self.R, dtype=np.int64)
        out = np.zeros((self.R, self.n), dtype=np.int8) if return_spins else None
        sp = None
        if spins is not None:
            sp = np.ascontiguousarray(spins, dtype=np.int8).reshape(self.R, self.n)
        _check(load_library().cosm_energy(self._h_state, _ptr(sp), _ptr(out), _ptr(H), _ptr(cut)))
        return H, cut, out

    def solve_to_target(self, target_H: int, max_trials: int, stop_at_first_hit=False):
        res = _CTTS()
        best = np.zeros(self.n, dtype=np.int8)
        _check(load_library().cosm_solve_to_target(self._h_state, int(target_H), int(max_trials),
                                                   int(bool(stop_at_first_hit)),
                                                   ctypes.byref(res), _ptr(best)))
        return TTSResult(*(getattr(res, f) for f, _ in _CTTS._fields_)), best

    def get_phases(self, unit=UNIT_TURNS):
        out = np.zeros((self.R, self.n), dtype=np.float64)
        _check(load_library().cosm_get_phases(self._h_state, int(unit), _ptr(out)))
        return out

    def set_phases(self, x, unit=UNIT_TURNS, t=0):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(self.R, self.n)
        _check(load_library().cosm_set_phases(self._h_state, int(unit), _ptr(x), int(t)))

    def info(self) -> dict:
        c = _CInfo()
        _check(load_library().cosm_get_info(self._h_state, ctypes.byref(c)))
        return {f: getattr(c, f) for f, _ in _CInfo._fields_}

    def set_timing(self, on: bool):
        _check(load_library().cosm_set_timing(self._h_state, int(bool(on))))


class Batch:
    """A cosm_batch: instances of uneven sizes run as whole trials by one
    persistent sweep launch (init, sweeps and readout replayed from a hipGraph).
    Runs on a torch stream of its own (graphs cannot be captured on the default
    stream)."""

    def __init__(self, storage=STORE_FP32, max_graphs=256, max_n=20000, max_bisectors=100):
        import torch
        L = load_library()
        if not torch.cuda.is_available():
            raise CosmError(-6, "no HIP device is visible")
        self._stream = torch.cuda.Stream()
        self.storage = storage
        h = ctypes.c_void_p()
        _check(L.cosm_batch_create(ctypes.byref(h), int(storage), int(max_graphs), int(max_n),
                                   int(max_bisectors), ctypes.c_void_p(self._stream.cuda_stream)))
        self._b = h
        self._sizes = []
        self._keep = []

    def add(self, n, eu, ev, J, colour, num_colours, params: Params, seed=0, replicas=1):
        eu, ev, J, colour = _i32(eu), _i32(ev), _i32(J), _i32(colour)
        gid = ctypes.c_int32(0)
        cp = params._c()
        _check(load_library().cosm_batch_add_graph(
            self._b, int(n), len(eu), _ptr(eu), _ptr(ev), _ptr(J), _ptr(colour), int(num_colours),
            ctypes.byref(cp), int(seed) & ((1 << 64) - 1), int(replicas), ctypes.byref(gid)))
        self._sizes.append((int(n), int(replicas)))
        return int(gid.value)

    def shape(self, graph_id):
        """replicas per set, sets per work item, how they were chosen (0: one
        width fits or was requested, 1: timed probes, 2: the probe cache), the
        chosen width's probe time in ms, and whether the phases are wrapped at
        the twists only."""
        rw, sets, tuned = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
        ms, lazy = ctypes.c_double(0.0), ctypes.c_int32(0)
        _check(load_library().cosm_batch_graph_shape(self._b, int(graph_id), ctypes.byref(rw),
                                                     ctypes.byref(sets), ctypes.byref(tuned),
                                                     ctypes.byref(ms), ctypes.byref(lazy)))
        return {"replicas_per_set": rw.value, "sets_per_item": sets.value, "tuned": tuned.value,
                "probe_ms": ms.value, "lazy_wrap": lazy.value}

    def set_seed(self, graph_id, seed, replica_offset=0):
        _check(load_library().cosm_batch_set_seed(self._b, int(graph_id),
                                                  int(seed) & ((1 << 64) - 1), int(replica_offset)))

    def run(self, graph_ids):
        ids = _i32(graph_ids)
        _check(load_library().cosm_batch_run(self._b, _ptr(ids), len(ids)))

    def wait(self):
        ms = ctypes.c_double(0.0)
        _check(load_library().cosm_batch_wait(self._b, ctypes.byref(ms)))
        return float(ms.value)

    def poll(self):
        """True once the last run has finished on the device (never blocks)."""
        done = ctypes.c_int32(0)
        _check(load_library().cosm_batch_poll(self._b, ctypes.byref(done)))
        return bool(done.value)

    def results(self, graph_id, return_spins=False):
        n, R = self._sizes[graph_id]
        H = np.zeros(R, dtype=np.int64)
        cut = np.zeros(R, dtype=np.int64)
        sp = np.zeros((R, n), dtype=np.int8) if return_spins else None
        _check(load_library().cosm_batch_results(self._b, int(graph_id), _ptr(H), _ptr(cut),
                                                 _ptr(sp)))
        return H, cut, sp

    def close(self):
        if getattr(self, "_b", None):
            load_library().cosm_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
