"""ctypes binding of libgp.so -- argument marshalling only.

Every computation runs inside the library (host C++ for generation and
validation, HIP kernels for evaluation, fitness, selection and gradients).
PyTorch supplies device memory and the current stream.  If the library is
missing this module raises at import: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgp.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
        "or `python -m paper_2110_11226_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

# ---- constants mirrored from include/gp.h ----
OP_VAR, OP_CONST, OP_ADD, OP_SUB, OP_MUL, OP_DIV, OP_NEG, OP_LOG, OP_SQRT, OP_SIN, OP_COS, OP_TAN = range(12)
OP_MAX, OP_MIN, OP_ATAN2 = 12, 13, 14
OP_ABS, OP_EXP, OP_INV, OP_SQ, OP_CUBE, OP_TANH, OP_ATAN, OP_CBRT = range(15, 23)
FUNCS_ALL = sum(1 << op for op in range(OP_ADD, OP_CBRT + 1))
OP_USER1, OP_USER2 = 24, 28   # user functions: 24..27 of one argument, 28..31 of two
MAX_STACK = 20
USER_MAX_NODES, USER_MAX_CONSTS, USER_MAX_STACK = 32, 16, 6
FUNCS_DEFAULT = 0x7FC
METRICS = {"mae": 0, "mse": 1, "rmse": 2, "logloss": 3, "pearson": 4, "spearman": 5,
           "user0": 6, "user1": 7, "user2": 8, "user3": 9}
INIT = {"rhh": 0, "full": 1, "grow": 2, "exact_len": 3}
STATUS = {0: "GP_OK", -1: "GP_ERR_INVALID_ARG", -2: "GP_ERR_INVALID_PROGRAM",
          -3: "GP_ERR_STACK_OVERFLOW", -4: "GP_ERR_OUT_OF_MEMORY", -5: "GP_ERR_DEVICE",
          -6: "GP_ERR_UNSUPPORTED", -7: "GP_ERR_BUFFER_TOO_SMALL"}

_vp = ctypes.c_void_p
_i32, _i64, _u32, _u64, _f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_float


class InitParams(ctypes.Structure):
    _fields_ = [("n_programs", _i32), ("n_features", _i32), ("method", _i32),
                ("min_depth", _i32), ("max_depth", _i32), ("min_len", _i32), ("max_len", _i32),
                ("function_mask", _u32), ("const_lo", _f32), ("const_hi", _f32),
                ("max_consts", _i32), ("seed", _u64)]


class PopulationDev(ctypes.Structure):
    _fields_ = [("nodes", _vp), ("prog_off", _vp), ("consts", _vp), ("const_off", _vp),
                ("len", _vp), ("n_programs", _i32), ("total_nodes", _i64), ("max_len", _i32),
                ("total_consts", _i64)]


class DatasetDev(ctypes.Structure):
    _fields_ = [("X", _vp), ("ld", _i64), ("n_features", _i32), ("n_rows", _i64),
                ("y", _vp), ("w", _vp)]


def _sig(name, args, res=ctypes.c_int):
    f = getattr(_lib, name)
    f.argtypes = args
    f.restype = res
    return f


_last_error = _sig("gp_last_error", [], ctypes.c_char_p)
_version = _sig("gp_version", [], ctypes.c_char_p)
_shutdown = _sig("gp_shutdown", [], None)
_larger = _sig("gp_metric_larger_is_better", [ctypes.c_int])
_build_pop = _sig("gp_build_population", [ctypes.POINTER(InitParams), _vp, _i64, _vp, _vp, _i64, _vp,
                                          _vp, _vp, _vp])
_validate = _sig("gp_validate_population", [_vp, _vp, _vp, _i32, _i32, _vp, _vp])
_evaluate = _sig("gp_evaluate", [ctypes.POINTER(PopulationDev), ctypes.POINTER(DatasetDev), _vp, _vp])
_fitness = _sig("gp_fitness", [ctypes.POINTER(PopulationDev), ctypes.POINTER(DatasetDev), ctypes.c_int,
                               _vp, _vp])
_fitness_noalloc = _sig("gp_fitness_noalloc", [ctypes.POINTER(PopulationDev), ctypes.POINTER(DatasetDev),
                                                ctypes.c_int, _vp, _vp])
_register_fn = _sig("gp_register_function", [_u32, _vp, _i32, _vp, _i32])
_fn_defined = _sig("gp_function_defined", [_u32])
_tournament = _sig("gp_tournament", [_vp, _vp, _i32, ctypes.c_int, _f32, _i32, _i32, _u64, _u64, _vp, _vp])
class LaunchConfig(ctypes.Structure):
    _fields_ = [("rows_per_lane", _i32), ("feature_regs", _i32), ("tiles_per_chunk", _i32),
                ("waves_per_block", _i32)]


_get_cfg = _sig("gp_get_launch_config", [_i32, _i64, _i32, ctypes.c_int, ctypes.POINTER(LaunchConfig)])
_set_cfg = _sig("gp_set_launch_config", [ctypes.POINTER(LaunchConfig)])
_set_spear_ws = _sig("gp_set_spearman_workset", [_i64])
_autotune = _sig("gp_autotune", [ctypes.POINTER(PopulationDev), ctypes.POINTER(DatasetDev), ctypes.c_int, _i32,
                                  ctypes.POINTER(LaunchConfig), ctypes.POINTER(ctypes.c_double), _vp])
_tune_save = _sig("gp_autotune_save", [ctypes.c_char_p])
_tune_load = _sig("gp_autotune_load", [ctypes.c_char_p])
_tune_clear = _sig("gp_autotune_clear", [])


class GenerationParams(ctypes.Structure):
    _fields_ = [("n_programs", _i32), ("node_capacity", _i64), ("const_capacity", _i64), ("metric", _i32),
                ("parsimony", _f32), ("tournament_size", _i32), ("n_tournaments", _i32), ("seed", _u64),
                ("autotune", _i32), ("time_kernel", _i32)]


_gen_create = _sig("gp_generation_create", [ctypes.POINTER(GenerationParams), ctypes.POINTER(DatasetDev),
                                            ctypes.POINTER(_vp)])
_gen_run = _sig("gp_generation_run", [_vp, _vp, _vp, _vp, _vp, _vp, _u64, _vp, _vp])
_gen_info = _sig("gp_generation_info", [_vp, ctypes.POINTER(LaunchConfig), ctypes.POINTER(_f32),
                                        ctypes.POINTER(_f32), ctypes.POINTER(_i32), ctypes.POINTER(ctypes.c_double)])
_gen_destroy = _sig("gp_generation_destroy", [_vp], None)


class EvolveParams(ctypes.Structure):
    _fields_ = [("p_crossover", _f32), ("p_subtree", _f32), ("p_hoist", _f32), ("p_point", _f32),
                ("p_point_replace", _f32), ("max_len", _i32), ("seed", _u64)]


_plan = _sig("gp_plan_generation", [ctypes.POINTER(EvolveParams), _i32, _u64, _vp, _vp, _vp])


class PopulationOutDev(ctypes.Structure):
    _fields_ = [("nodes", _vp), ("prog_off", _vp), ("consts", _vp), ("const_off", _vp), ("len", _vp),
                ("node_capacity", _i64), ("const_capacity", _i64)]


_plan_dev = _sig("gp_plan_generation_device", [ctypes.POINTER(EvolveParams), _i32, _u64, _vp, _vp, _vp, _vp])
_mutate_dev = _sig("gp_mutate_device", [ctypes.POINTER(EvolveParams), ctypes.POINTER(InitParams),
                                        ctypes.POINTER(PopulationDev), _vp, _vp, _vp, _i32, _i32, _u64,
                                        ctypes.POINTER(PopulationOutDev), _vp, _vp])
_mutate = _sig("gp_mutate", [ctypes.POINTER(EvolveParams), ctypes.POINTER(InitParams), _vp, _vp, _vp, _vp, _i32,
                             _vp, _vp, _vp, _i32, _i32, _u64, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _vp, _vp])
GENOPS = {"crossover": 0, "subtree": 1, "hoist": 2, "point": 3, "reproduction": 4}
class Profile(ctypes.Structure):
    _fields_ = [("launches", _i64), ("total_ms", ctypes.c_double), ("node_rows", _i64)]


_prof_enable = _sig("gp_profile_enable", [ctypes.c_int])
_prof_read = _sig("gp_profile_read", [ctypes.POINTER(Profile)])
_backward = _sig("gp_fitness_backward", [ctypes.POINTER(PopulationDev), ctypes.POINTER(DatasetDev),
                                         ctypes.c_int, _vp, _vp, _vp, _vp])

EXPORTED = ["gp_last_error", "gp_version", "gp_shutdown", "gp_metric_larger_is_better",
            "gp_build_population", "gp_validate_population", "gp_evaluate", "gp_fitness", "gp_fitness_noalloc",
            "gp_register_function", "gp_function_defined",
            "gp_tournament", "gp_fitness_backward", "gp_get_launch_config", "gp_set_launch_config",
            "gp_profile_enable", "gp_profile_read", "gp_autotune", "gp_autotune_save", "gp_autotune_load",
            "gp_autotune_clear", "gp_generation_create", "gp_generation_run", "gp_generation_info",
            "gp_generation_destroy", "gp_plan_generation", "gp_mutate"]


def profile_enable(on=True):
    _check(_prof_enable(1 if on else 0), "gp_profile_enable")


def profile_read():
    """(launches, total_ms, node_rows) of the evaluation kernel since enabled."""
    p = Profile()
    _check(_prof_read(ctypes.byref(p)), "gp_profile_read")
    return int(p.launches), float(p.total_ms), int(p.node_rows)


def get_launch_config(n_features, n_rows, n_programs, metric="mse"):
    c = LaunchConfig()
    _check(_get_cfg(n_features, n_rows, n_programs, metric_id(metric), ctypes.byref(c)), "gp_get_launch_config")
    return (c.rows_per_lane, c.feature_regs, c.tiles_per_chunk, c.waves_per_block)


def autotune(pop, data, metric="mse", repeats=2, stream=None):
    """Times candidate launch configurations (see gp_autotune); returns
    ((rows_per_lane, feature_regs, tiles_per_chunk), best_ms)."""
    c = LaunchConfig()
    ms = ctypes.c_double(-1.0)
    _check(_autotune(ctypes.byref(pop.view), ctypes.byref(data.view), metric_id(metric), int(repeats),
                     ctypes.byref(c), ctypes.byref(ms), _stream(stream)), "gp_autotune")
    return (c.rows_per_lane, c.feature_regs, c.tiles_per_chunk, c.waves_per_block), float(ms.value)


def autotune_save(path):
    _check(_tune_save(os.fsencode(path)), "gp_autotune_save")


def autotune_load(path):
    _check(_tune_load(os.fsencode(path)), "gp_autotune_load")


def autotune_clear():
    _check(_tune_clear(), "gp_autotune_clear")


def set_launch_config(cfg=None):
    """cfg = (rows_per_lane, feature_regs, tiles_per_chunk[, waves_per_block
    = 4]) or None for automatic."""
    if cfg is None:
        _check(_set_cfg(None), "gp_set_launch_config")
    else:
        v = [int(x) for x in cfg]
        if len(v) == 3:
            v.append(4)
        c = LaunchConfig(*v)
        _check(_set_cfg(ctypes.byref(c)), "gp_set_launch_config")


def set_spearman_workset(max_bytes=0):
    """Device memory Spearman fitness may use for a batch of programs (16
    bytes per row per program); 0 returns to the default (16 GiB, at most half
    the free memory)."""
    _check(_set_spear_ws(int(max_bytes)), "gp_set_spearman_workset")


class GPError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")


def _check(rc: int, where: str):
    if rc != 0:
        raise GPError(rc, where)


def version() -> str:
    return _version().decode()


def shutdown():
    _shutdown()


def metric_id(metric) -> int:
    return METRICS[metric] if isinstance(metric, str) else int(metric)


def larger_is_better(metric) -> bool:
    return bool(_larger(metric_id(metric)))


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(_vp)


# ---------------------------------------------------------------------------
# Host population
# ---------------------------------------------------------------------------
@dataclass
class HostPopulation:
    nodes: np.ndarray      # uint32
    prog_off: np.ndarray   # int64 [P+1]
    consts: np.ndarray     # float32
    const_off: np.ndarray  # int64 [P+1]
    length: np.ndarray     # int32 [P]

    @property
    def n_programs(self) -> int:
        return int(self.length.shape[0])


def build_population(n_programs, n_features, method="rhh", min_depth=2, max_depth=6, min_len=1,
                     max_len=200, function_mask=FUNCS_DEFAULT, const_lo=-1.0, const_hi=1.0,
                     max_consts=0, seed=0) -> HostPopulation:
    prm = InitParams(n_programs, n_features, INIT[method] if isinstance(method, str) else int(method),
                     min_depth, max_depth, min_len, max_len, function_mask, const_lo, const_hi,
                     max_consts, seed)
    tn = np.zeros(1, np.int64)
    tc = np.zeros(1, np.int64)
    _check(_build_pop(ctypes.byref(prm), None, 0, None, None, 0, None, None, _np_ptr(tn), _np_ptr(tc)),
           "gp_build_population")
    nodes = np.zeros(max(int(tn[0]), 1), np.uint32)
    consts = np.zeros(max(int(tc[0]), 1), np.float32)
    po = np.zeros(n_programs + 1, np.int64)
    co = np.zeros(n_programs + 1, np.int64)
    ln = np.zeros(max(n_programs, 1), np.int32)
    _check(_build_pop(ctypes.byref(prm), _np_ptr(nodes), nodes.shape[0], _np_ptr(po), _np_ptr(consts),
                      consts.shape[0], _np_ptr(co), _np_ptr(ln), _np_ptr(tn), _np_ptr(tc)),
           "gp_build_population")
    return HostPopulation(nodes[:int(tn[0])], po, consts[:int(tc[0])], co, ln[:n_programs])


def validate_population(pop: HostPopulation, n_features: int):
    """Returns per-program peak stack heights; raises GPError if invalid."""
    P = pop.n_programs
    h = np.zeros(max(P, 1), np.int32)
    bad = np.full(1, -1, np.int32)
    nodes = np.ascontiguousarray(pop.nodes, np.uint32)
    rc = _validate(_np_ptr(nodes), _np_ptr(np.ascontiguousarray(pop.prog_off, np.int64)),
                   _np_ptr(np.ascontiguousarray(pop.const_off, np.int64)), P, n_features,
                   _np_ptr(h), _np_ptr(bad))
    _check(rc, "gp_validate_population")
    return h[:P]


# ---------------------------------------------------------------------------
# Device views (torch tensors on the current HIP device)
# ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _tptr(t):
    return None if t is None else _vp(t.data_ptr())


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return _vp(s.cuda_stream)


class DevicePopulation:
    """A flat population resident on the device (one contiguous upload)."""

    def __init__(self, host: HostPopulation, device="cuda", validate=True, n_features=None):
        torch = _torch()
        if validate:
            if n_features is None:
                raise ValueError("n_features is needed to validate")
            validate_population(host, n_features)
        self.host = host
        self.nodes = torch.from_numpy(np.ascontiguousarray(host.nodes, np.uint32).view(np.int32)).to(device)
        self.prog_off = torch.from_numpy(np.ascontiguousarray(host.prog_off, np.int64)).to(device)
        c = host.consts if host.consts.shape[0] else np.zeros(1, np.float32)
        self.consts = torch.from_numpy(np.ascontiguousarray(c, np.float32)).to(device)
        self.const_off = torch.from_numpy(np.ascontiguousarray(host.const_off, np.int64)).to(device)
        self.length = torch.from_numpy(np.ascontiguousarray(host.length, np.int32)).to(device)
        self.n_programs = host.n_programs
        self.n_consts = int(host.consts.shape[0])
        self.max_len = int(host.length.max()) if self.n_programs else 0
        self.view = self.make_view(self.consts)

    def make_view(self, consts):
        return PopulationDev(self.nodes.data_ptr(), self.prog_off.data_ptr(), consts.data_ptr(),
                             self.const_off.data_ptr(), self.length.data_ptr(), self.n_programs,
                             self.total_nodes, self.max_len, self.n_consts)

    @property
    def total_nodes(self):
        return int(self.host.nodes.shape[0]) if self.host is not None else self._total_nodes

    @classmethod
    def from_device(cls, nodes, prog_off, consts, const_off, length, total_nodes, total_consts, max_len):
        """A view of a population already on the device (offsets and
        lengths describe valid programs; max_len bounds every length)."""
        self = cls.__new__(cls)
        self.host = None
        self.nodes, self.prog_off, self.consts = nodes, prog_off, consts
        self.const_off, self.length = const_off, length
        self.n_programs = int(length.shape[0])
        self.n_consts = int(total_consts)
        self._total_nodes = int(total_nodes)
        self.max_len = int(max_len)
        self.view = self.make_view(self.consts)
        return self


class DeviceDataset:
    """Feature-major X[f, r], target y[r], optional weights w[r] on the device."""

    def __init__(self, X, y=None, w=None, device="cuda"):
        torch = _torch()

        def dev(a):
            if a is None:
                return None
            t = a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(a, np.float32))
            return t.to(device=device, dtype=torch.float32).contiguous()

        self.X = dev(X)
        self.y = dev(y)
        self.w = dev(w)
        self.n_features, self.n_rows = int(self.X.shape[0]), int(self.X.shape[1])
        self.view = DatasetDev(self.X.data_ptr(), self.n_rows, self.n_features, self.n_rows,
                               self.y.data_ptr() if self.y is not None else None,
                               self.w.data_ptr() if self.w is not None else None)


def evaluate(pop: DevicePopulation, data: DeviceDataset, out=None, stream=None):
    torch = _torch()
    if out is None:
        out = torch.empty((pop.n_programs, data.n_rows), dtype=torch.float32, device=data.X.device)
    _check(_evaluate(ctypes.byref(pop.view), ctypes.byref(data.view), _tptr(out), _stream(stream)),
           "gp_evaluate")
    return out


def fitness(pop: DevicePopulation, data: DeviceDataset, metric="mse", out=None, stream=None, consts=None):
    torch = _torch()
    if out is None:
        out = torch.empty(pop.n_programs, dtype=torch.float32, device=data.X.device)
    view = pop.view if consts is None else pop.make_view(consts)
    _check(_fitness(ctypes.byref(view), ctypes.byref(data.view), metric_id(metric), _tptr(out),
                    _stream(stream)), "gp_fitness")
    return out


def register_function(op, nodes=None, consts=()):
    """gp_register_function: define user function `op` (24..27: one
    argument, 28..31: two) as the prefix list `nodes` (node words over the
    built-in functions, OP_VAR k = argument k, OP_CONST k = consts[k]);
    nodes None or empty removes the definition."""
    if not nodes:
        _check(_register_fn(int(op), None, 0, None, 0), "gp_register_function")
        return
    nd = np.ascontiguousarray(np.asarray(nodes, np.uint32))
    cs = np.ascontiguousarray(np.asarray(consts, np.float32))
    _check(_register_fn(int(op), _np_ptr(nd), int(nd.shape[0]), _np_ptr(cs) if cs.size else None, int(cs.size)),
           "gp_register_function")


def function_defined(op) -> bool:
    return bool(_fn_defined(int(op)))


def fitness_noalloc(pop: DevicePopulation, data: DeviceDataset, metric="mse", out=None, stream=None):
    """gp_fitness_noalloc: fitness with the library's static device scratch
    (no device allocation inside the call; `out` may be preallocated)."""
    torch = _torch()
    if out is None:
        out = torch.empty(pop.n_programs, dtype=torch.float32, device=data.X.device)
    _check(_fitness_noalloc(ctypes.byref(pop.view), ctypes.byref(data.view), metric_id(metric), _tptr(out),
                            _stream(stream)), "gp_fitness_noalloc")
    return out


def tournament(fit, length, metric="mse", parsimony=0.0, tournament_size=20, n_tournaments=None,
               seed=0, generation=0, out=None, stream=None):
    torch = _torch()
    P = int(fit.shape[0])
    T = P if n_tournaments is None else int(n_tournaments)
    if out is None:
        out = torch.empty(max(T, 1), dtype=torch.int32, device=fit.device)
    _check(_tournament(_tptr(fit), _tptr(length), P, metric_id(metric), float(parsimony),
                       int(tournament_size), T, int(seed), int(generation), _tptr(out), _stream(stream)),
           "gp_tournament")
    return out[:T]


def fitness_backward(pop: DevicePopulation, data: DeviceDataset, metric="mse", grad_fitness=None,
                     consts=None, fitness_out=None, grad_out=None, stream=None):
    torch = _torch()
    c = pop.consts if consts is None else consts
    view = pop.view if consts is None else pop.make_view(c)
    if grad_out is None:
        grad_out = torch.zeros(max(pop.n_consts, 1), dtype=torch.float32, device=data.X.device)
    _check(_backward(ctypes.byref(view), ctypes.byref(data.view), metric_id(metric), _tptr(grad_fitness),
                     _tptr(fitness_out), _tptr(grad_out), _stream(stream)), "gp_fitness_backward")
    return grad_out[:pop.n_consts]


class Generation:
    """One generation as a captured HIP graph (gp_generation_*): upload of the
    host population, fitness, tournaments, download of fitness and winners."""

    def __init__(self, data: DeviceDataset, n_programs, node_capacity, const_capacity, metric="mse",
                 parsimony=0.0, tournament_size=20, n_tournaments=None, seed=0, autotune=False,
                 time_kernel=False):
        self.data = data          # the dataset must outlive the graph
        self.n_programs = int(n_programs)
        self.n_tournaments = self.n_programs if n_tournaments is None else int(n_tournaments)
        prm = GenerationParams(self.n_programs, int(node_capacity), int(const_capacity), metric_id(metric),
                               float(parsimony), int(tournament_size), self.n_tournaments, int(seed),
                               1 if autotune else 0, 1 if time_kernel else 0)
        h = _vp()
        _check(_gen_create(ctypes.byref(prm), ctypes.byref(data.view), ctypes.byref(h)), "gp_generation_create")
        self._h = h

    def run(self, pop: HostPopulation, generation):
        """(fitness float32 [P], winners int32 [T]) as numpy arrays."""
        if pop.n_programs != self.n_programs:
            raise ValueError("population size differs from the one the graph was built for")
        nodes = np.ascontiguousarray(pop.nodes, np.uint32)
        po = np.ascontiguousarray(pop.prog_off, np.int64)
        c = np.ascontiguousarray(pop.consts, np.float32)
        co = np.ascontiguousarray(pop.const_off, np.int64)
        ln = np.ascontiguousarray(pop.length, np.int32)
        fit = np.empty(self.n_programs, np.float32)
        win = np.empty(max(self.n_tournaments, 1), np.int32)
        _check(_gen_run(self._h, _np_ptr(nodes), _np_ptr(po), _np_ptr(c) if c.shape[0] else None, _np_ptr(co),
                        _np_ptr(ln), int(generation), _np_ptr(fit), _np_ptr(win)), "gp_generation_run")
        return fit, win[:self.n_tournaments]

    def info(self):
        """(launch configuration, kernel_ms of the last run, tuned_ms)."""
        d = self.timing()
        return d["launch"], d["kernel_ms"], d["tuned_ms"]

    def timing(self):
        """Launch configuration, the evaluation kernel's last duration (HIP
        event nodes if the graph holds them, else the device clock), the
        clock-stamp duration, which method timed it, and the tuned time."""
        c = LaunchConfig()
        k = _f32(-1.0)
        ck = _f32(-1.0)
        ev = _i32(0)
        t = ctypes.c_double(-1.0)
        _check(_gen_info(self._h, ctypes.byref(c), ctypes.byref(k), ctypes.byref(ck), ctypes.byref(ev),
                         ctypes.byref(t)), "gp_generation_info")
        return {"launch": (c.rows_per_lane, c.feature_regs, c.tiles_per_chunk, c.waves_per_block),
                "kernel_ms": float(k.value),
                "clock_ms": float(ck.value), "timed_by": "hip_events" if ev.value else "device_clock",
                "tuned_ms": float(t.value)}

    def close(self):
        if self._h:
            _gen_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _evolve_struct(p_crossover=0.7, p_subtree=0.1, p_hoist=0.05, p_point=0.1, p_point_replace=0.05,
                   max_len=4096, seed=0):
    return EvolveParams(p_crossover, p_subtree, p_hoist, p_point, p_point_replace, max_len, seed)


def _init_struct(n_features, method="rhh", min_depth=2, max_depth=6, min_len=1, max_len=200,
                 function_mask=FUNCS_DEFAULT, const_lo=-1.0, const_hi=1.0, max_consts=0, seed=0):
    return InitParams(0, n_features, INIT[method] if isinstance(method, str) else int(method), min_depth,
                      max_depth, min_len, max_len, function_mask, const_lo, const_hi, max_consts, seed)


def plan_generation(n_offspring, generation, **evolve):
    """(ops, first_tournament, n_tournaments): the operation of every
    offspring and where its tournaments start (gp_plan_generation)."""
    ev = _evolve_struct(**evolve)
    ops = np.zeros(max(n_offspring, 1), np.int32)
    ft = np.zeros(max(n_offspring, 1), np.int32)
    nt = np.zeros(1, np.int32)
    _check(_plan(ctypes.byref(ev), int(n_offspring), int(generation), _np_ptr(ops), _np_ptr(ft), _np_ptr(nt)),
           "gp_plan_generation")
    return ops[:n_offspring], ft[:n_offspring], int(nt[0])


def mutate(parents: HostPopulation, ops, first_tournament, winners, generation, init: dict, **evolve):
    """The offspring population (gp_mutate).  init: the initialisation
    settings (n_features, method, depths/lengths, function_mask, constants)
    that donors of subtree mutation follow."""
    ev = _evolve_struct(**evolve)
    ip = _init_struct(**init)
    n_off = int(len(ops))
    ops = np.ascontiguousarray(ops, np.int32)
    ft = np.ascontiguousarray(first_tournament, np.int32)
    win = np.ascontiguousarray(winners, np.int32)
    longest = int(parents.length.max(initial=1))
    cap = max(n_off * max(int(ev.max_len), longest, 1), 1)
    nodes = np.zeros(cap, np.uint32)
    consts = np.zeros(cap, np.float32)
    po = np.zeros(n_off + 1, np.int64)
    co = np.zeros(n_off + 1, np.int64)
    ln = np.zeros(max(n_off, 1), np.int32)
    tn = np.zeros(1, np.int64)
    tc = np.zeros(1, np.int64)
    pn = np.ascontiguousarray(parents.nodes, np.uint32)
    pc = np.ascontiguousarray(parents.consts if parents.consts.shape[0] else np.zeros(1, np.float32), np.float32)
    args = [ctypes.byref(ev), ctypes.byref(ip), _np_ptr(pn), _np_ptr(np.ascontiguousarray(parents.prog_off, np.int64)),
            _np_ptr(pc), _np_ptr(np.ascontiguousarray(parents.const_off, np.int64)), parents.n_programs,
            _np_ptr(ops), _np_ptr(ft), _np_ptr(win), int(win.shape[0]), n_off, int(generation)]
    rc = _mutate(*args, _np_ptr(nodes), cap, _np_ptr(po), _np_ptr(consts), cap, _np_ptr(co), _np_ptr(ln),
                 _np_ptr(tn), _np_ptr(tc))
    if rc == -7:   # GP_ERR_BUFFER_TOO_SMALL: retry at the reported size
        nodes = np.zeros(max(int(tn[0]), 1), np.uint32)
        consts = np.zeros(max(int(tc[0]), 1), np.float32)
        rc = _mutate(*args, _np_ptr(nodes), nodes.shape[0], _np_ptr(po), _np_ptr(consts), consts.shape[0],
                     _np_ptr(co), _np_ptr(ln), _np_ptr(tn), _np_ptr(tc))
    _check(rc, "gp_mutate")
    return HostPopulation(nodes[:int(tn[0])].copy(), po, consts[:int(tc[0])].copy(), co, ln[:n_off].copy())



def plan_generation_device(n_offspring, generation, stream=None, **evolve):
    """(ops, first_tournament, n_tournaments) as DEVICE int32 tensors
    ([n_offspring], [n_offspring], [1]); gp_plan_generation_device."""
    torch = _torch()
    ev = _evolve_struct(**evolve)
    n = int(n_offspring)
    ops = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    ft = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    nt = torch.empty(1, dtype=torch.int32, device="cuda")
    _check(_plan_dev(ctypes.byref(ev), n, int(generation), _tptr(ops), _tptr(ft), _tptr(nt), _stream(stream)),
           "gp_plan_generation_device")
    return ops[:n], ft[:n], nt


MUTATE_STATUS = {1: "a capacity of the output is short; nothing was written",
                 2: "an operation, tournament or winner index was out of range",
                 4: "the subtree-mutation donors overflowed the library's bound"}


class DeviceOffspring:
    """An offspring population written on the device by gp_mutate_device."""

    def __init__(self, nodes, prog_off, consts, const_off, length, info, max_len):
        self.nodes, self.prog_off, self.consts = nodes, prog_off, consts
        self.const_off, self.length, self.info = const_off, length, info
        self.max_len = int(max_len)

    def status(self):
        """(total_nodes, total_consts, status bits) after synchronising."""
        v = self.info.cpu().numpy()
        return int(v[0]), int(v[1]), int(v[2])

    def check(self):
        tn, tc, st = self.status()
        if st:
            msgs = [m for b, m in MUTATE_STATUS.items() if st & b]
            raise GPError(-1, "gp_mutate_device: " + "; ".join(msgs))
        return tn, tc

    def to_host(self) -> HostPopulation:
        tn, tc = self.check()
        return HostPopulation(self.nodes[:tn].cpu().numpy().view(np.uint32).copy(),
                              self.prog_off.cpu().numpy().copy(), self.consts[:tc].cpu().numpy().copy(),
                              self.const_off.cpu().numpy().copy(), self.length.cpu().numpy().copy())

    def as_parents(self) -> DevicePopulation:
        """This population as the next generation's device parents (reads the
        totals, so it synchronises)."""
        tn, tc = self.check()
        return DevicePopulation.from_device(self.nodes, self.prog_off, self.consts, self.const_off, self.length,
                                            tn, tc, self.max_len)


def mutate_device(parents: DevicePopulation, ops, first_tournament, winners, generation, init: dict,
                  stream=None, node_capacity=None, const_capacity=None, **evolve) -> DeviceOffspring:
    """The offspring population on the device (gp_mutate_device); ops,
    first_tournament and winners are device int32 tensors (or arrays,
    uploaded).  The default capacities hold any outcome: every child is at
    most max(max_len, the longest parent) nodes long."""
    torch = _torch()
    ev = _evolve_struct(**evolve)
    ip = _init_struct(**init)

    def dev_i32(a):
        t = a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(a, np.int32))
        return t.to(device="cuda", dtype=torch.int32).contiguous()

    ops, ft, win = dev_i32(ops), dev_i32(first_tournament), dev_i32(winners)
    n_off = int(ops.shape[0])
    longest = max(int(ev.max_len), int(parents.max_len), 1)
    ncap = int(node_capacity) if node_capacity is not None else max(n_off * longest, 1)
    ccap = int(const_capacity) if const_capacity is not None else max(n_off * longest, 1)
    nodes = torch.empty(max(ncap, 1), dtype=torch.int32, device="cuda")
    consts = torch.empty(max(ccap, 1), dtype=torch.float32, device="cuda")
    po = torch.empty(n_off + 1, dtype=torch.int64, device="cuda")
    co = torch.empty(n_off + 1, dtype=torch.int64, device="cuda")
    ln = torch.empty(max(n_off, 1), dtype=torch.int32, device="cuda")
    info = torch.empty(4, dtype=torch.int64, device="cuda")
    out = PopulationOutDev(nodes.data_ptr(), po.data_ptr(), consts.data_ptr(), co.data_ptr(), ln.data_ptr(),
                           ncap, ccap)
    _check(_mutate_dev(ctypes.byref(ev), ctypes.byref(ip), ctypes.byref(parents.view), _tptr(ops), _tptr(ft),
                       _tptr(win), int(win.shape[0]), n_off, int(generation), ctypes.byref(out), _tptr(info),
                       _stream(stream)), "gp_mutate_device")
    return DeviceOffspring(nodes, po, consts, co, ln[:n_off], info, longest)


class EvolutionParams(ctypes.Structure):
    _fields_ = [("n_programs", _i32), ("metric", _i32), ("parsimony", _f32), ("tournament_size", _i32),
                ("tournament_seed", _u64), ("evolve", EvolveParams), ("init", InitParams),
                ("max_generations", _i32), ("autotune", _i32), ("time_kernel", _i32),
                ("first_generation", _u64)]


_evo_create = _sig("gp_evolution_create", [ctypes.POINTER(EvolutionParams), ctypes.POINTER(DatasetDev), _vp, _vp,
                                           _vp, _vp, _vp, ctypes.POINTER(_vp)])
_evo_run = _sig("gp_evolution_run", [_vp, _i32])
_evo_eval = _sig("gp_evolution_evaluate", [_vp])
_evo_hist = _sig("gp_evolution_history", [_vp, _i32, _vp, _vp, _vp])
_evo_pop = _sig("gp_evolution_population", [_vp, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _vp, _vp])
_evo_info = _sig("gp_evolution_info", [_vp, ctypes.POINTER(LaunchConfig), ctypes.POINTER(_f32),
                                       ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_double)])
_evo_destroy = _sig("gp_evolution_destroy", [_vp], None)


class Evolution:
    """The device-resident generational loop (gp_evolution_*): each generation
    is one graph replay -- fitness, history record, tournaments, operation
    pre-draw, genetic operations -- with no host round trip."""

    def __init__(self, data: DeviceDataset, pop: HostPopulation, init: dict, evolve: dict | None = None,
                 metric="mse", parsimony=0.0, tournament_size=20, tournament_seed=0, max_generations=100,
                 autotune=False, time_kernel=False, first_generation=0):
        self.data = data
        self.n_programs = pop.n_programs
        ev = _evolve_struct(**(evolve or {}))
        ip = _init_struct(**init)
        prm = EvolutionParams(self.n_programs, metric_id(metric), float(parsimony), int(tournament_size),
                              int(tournament_seed), ev, ip, int(max_generations), int(bool(autotune)),
                              int(bool(time_kernel)), int(first_generation))
        c = pop.consts if pop.consts.shape[0] else np.zeros(1, np.float32)
        self._keep = [np.ascontiguousarray(pop.nodes, np.uint32), np.ascontiguousarray(pop.prog_off, np.int64),
                      np.ascontiguousarray(c, np.float32), np.ascontiguousarray(pop.const_off, np.int64),
                      np.ascontiguousarray(pop.length, np.int32)]
        h = _vp()
        _check(_evo_create(ctypes.byref(prm), ctypes.byref(data.view), *[_np_ptr(a) for a in self._keep],
                           ctypes.byref(h)), "gp_evolution_create")
        self._h = h
        self._keep = None

    def run(self, n_generations):
        _check(_evo_run(self._h, int(n_generations)), "gp_evolution_run")

    def evaluate(self):
        _check(_evo_eval(self._h), "gp_evolution_evaluate")

    def history(self):
        """(fitness [n_recorded, n_programs], total nodes [n_recorded])."""
        n = _i32()
        _check(_evo_hist(self._h, 0, ctypes.byref(n), None, None), "gp_evolution_history")
        k = int(n.value)
        fit = np.zeros((max(k, 1), self.n_programs), np.float32)
        nodes = np.zeros(max(k, 1), np.int64)
        _check(_evo_hist(self._h, k, ctypes.byref(n), _np_ptr(fit), _np_ptr(nodes)), "gp_evolution_history")
        return fit[:k], nodes[:k]

    def population(self) -> HostPopulation:
        P = self.n_programs
        po = np.zeros(P + 1, np.int64)
        co = np.zeros(P + 1, np.int64)
        ln = np.zeros(P, np.int32)
        tn, tc = _i64(), _i64()
        rc = _evo_pop(self._h, None, 0, _np_ptr(po), None, 0, _np_ptr(co), _np_ptr(ln), ctypes.byref(tn),
                      ctypes.byref(tc))
        if rc not in (0, -7):
            _check(rc, "gp_evolution_population")
        nodes = np.zeros(max(tn.value, 1), np.uint32)
        consts = np.zeros(max(tc.value, 1), np.float32)
        _check(_evo_pop(self._h, _np_ptr(nodes), nodes.shape[0], _np_ptr(po), _np_ptr(consts), consts.shape[0],
                        _np_ptr(co), _np_ptr(ln), ctypes.byref(tn), ctypes.byref(tc)), "gp_evolution_population")
        return HostPopulation(nodes[:tn.value].copy(), po, consts[:tc.value].copy(), co, ln)

    def info(self):
        """(launch config tuple, evaluation-kernel ms of the last replay (-1
        if not timed), generations run, autotuner best ms (-1 if not tuned))."""
        cfg = LaunchConfig()
        ms = _f32()
        g = _i64()
        t = ctypes.c_double()
        _check(_evo_info(self._h, ctypes.byref(cfg), ctypes.byref(ms), ctypes.byref(g), ctypes.byref(t)),
               "gp_evolution_info")
        return ((cfg.rows_per_lane, cfg.feature_regs, cfg.tiles_per_chunk, cfg.waves_per_block), float(ms.value),
                int(g.value), float(t.value))

    def close(self):
        if getattr(self, "_h", None):
            _evo_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
