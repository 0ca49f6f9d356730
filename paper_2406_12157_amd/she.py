"""ctypes binding of libshe (include/she.h): argument marshalling only.

Every step of the method runs in the HIP kernels of libshe.so.  PyTorch is
used for device memory (an optional arena tensor) and for the stream the
library enqueues on.  If the library has not been built the import of this
module raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libshe.so")

HEAT, SPECIES, BURGERS = 0, 1, 2
PERIODIC, DIRICHLET = 0, 1
EM, HEUN, BE, CN = 0, 1, 2, 3
NOISE_INSTANT, NOISE_FROZEN, NOISE_OFF = 0, 1, 2
F32, F64 = 0, 1
STAT_MOMENTS, STAT_CORR, STAT_SK, STAT_SPATIAL, STAT_TCORR = 1, 2, 4, 8, 16
TUNE_XCD_ORDER = 1
TUNE_SEARCH = 2
TUNE_SINGLE_STEP = 4
ALLOW_UNSTABLE = 1

OK, EINVAL, EUNSTABLE, ENOMEM, EDEVICE, ENONFINITE, ESTATE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
_NAMES = {0: "SHE_OK", -1: "SHE_EINVAL", -2: "SHE_EUNSTABLE", -3: "SHE_ENOMEM", -4: "SHE_EDEVICE",
          -5: "SHE_ENONFINITE", -6: "SHE_ESTATE", -7: "SHE_EUNSUPPORTED"}


class SheError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_NAMES.get(status, str(status)), msg))
        self.status = status


class InstanceDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3), ("eq", C.c_int32), ("bc", C.c_int32),
                ("scheme", C.c_int32), ("noise", C.c_int32), ("r", C.c_double), ("eps", C.c_double),
                ("u0", C.c_double), ("u_left", C.c_double), ("u_right", C.c_double),
                ("init_sd", C.c_double), ("seed", C.c_uint64), ("realisation", C.c_uint32),
                ("reserved", C.c_uint32), ("cond", C.POINTER(C.c_double)), ("cap", C.POINTER(C.c_double)),
                ("nu", C.c_double)]


class Config(C.Structure):
    _fields_ = [("n_instances", C.c_int32), ("precision", C.c_int32), ("inst", C.POINTER(InstanceDesc)),
                ("burn_in", C.c_int64), ("sample_every", C.c_int32), ("stats_mask", C.c_uint32),
                ("block_threads", C.c_int32), ("rows_per_block", C.c_int32), ("rows_per_group", C.c_int32),
                ("tuning_flags", C.c_int32), ("graph_steps", C.c_int32), ("tcorr_lags", C.c_int32),
                ("batch_samples", C.c_int32), ("flags", C.c_uint32),
                ("stream", C.c_void_p), ("arena", C.c_void_p),
                ("arena_bytes", C.c_size_t)]


class StatsOut(C.Structure):
    _fields_ = [("n_samples", C.c_int64), ("steps", C.c_int64),
                ("mean", C.POINTER(C.c_double)), ("mean_cap", C.c_int64),
                ("var", C.POINTER(C.c_double)), ("var_cap", C.c_int64),
                ("corr", C.POINTER(C.c_double)), ("corr_cap", C.c_int64),
                ("sk", C.POINTER(C.c_double)), ("sk_cap", C.c_int64),
                ("sk_modes", C.POINTER(C.c_double)), ("sk_modes_cap", C.c_int64),
                ("sum_u", C.c_double), ("nonfinite", C.c_int32), ("reserved", C.c_int32),
                ("clamp_count", C.c_int64), ("tcorr", C.POINTER(C.c_double)), ("tcorr_cap", C.c_int64),
                ("n_batches", C.c_int64),
                ("mean_se", C.POINTER(C.c_double)), ("mean_se_cap", C.c_int64),
                ("var_se", C.POINTER(C.c_double)), ("var_se_cap", C.c_int64),
                ("sk_se", C.POINTER(C.c_double)), ("sk_se_cap", C.c_int64),
                ("spatial_var", C.c_double), ("spatial_var_se", C.c_double)]


EXPORTS = ["she_create", "she_arena_bytes", "she_tune", "she_step", "she_run", "she_stats", "she_reset_stats",
           "she_read_field", "she_write_field", "she_get_step", "she_state_bytes", "she_get_state",
           "she_set_state", "she_last_error", "she_destroy", "she_debug_philox", "she_debug_normals",
           "she_debug_normals_noalloc"]
NOALLOC_MAX_NORMALS = 1 << 20

_lib = None


def load(path: str = LIB_PATH):
    """Load libshe.so and declare its signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libshe.so not built at %s; run __graft_entry__.build()" % path)
    lib = C.CDLL(path)
    P = C.POINTER
    lib.she_create.argtypes = [P(Config), P(C.c_void_p)]
    lib.she_arena_bytes.argtypes = [P(Config), P(C.c_size_t)]
    lib.she_tune.argtypes = [P(Config), C.c_int32, P(Config)]
    lib.she_step.argtypes = [C.c_void_p, C.c_int64]
    lib.she_run.argtypes = [C.c_void_p, C.c_int64]
    lib.she_stats.argtypes = [C.c_void_p, C.c_int32, P(StatsOut)]
    lib.she_reset_stats.argtypes = [C.c_void_p]
    lib.she_read_field.argtypes = [C.c_void_p, C.c_int32, P(C.c_double), C.c_int64]
    lib.she_write_field.argtypes = [C.c_void_p, C.c_int32, P(C.c_double), C.c_int64]
    lib.she_get_step.argtypes = [C.c_void_p, P(C.c_int64)]
    lib.she_state_bytes.argtypes = [C.c_void_p, P(C.c_size_t)]
    lib.she_get_state.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
    lib.she_set_state.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
    lib.she_last_error.argtypes = [C.c_void_p]
    lib.she_last_error.restype = C.c_char_p
    lib.she_destroy.argtypes = [C.c_void_p]
    lib.she_destroy.restype = None
    lib.she_debug_philox.argtypes = [C.c_uint64, P(C.c_uint32), C.c_int64, P(C.c_uint32), C.c_void_p]
    lib.she_debug_normals.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint64, C.c_int64,
                                      C.c_int32, P(C.c_double), C.c_void_p]
    lib.she_debug_normals_noalloc.argtypes = lib.she_debug_normals.argtypes
    for name in EXPORTS:
        if name not in ("she_last_error", "she_destroy"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(status: int, handle=None):
    if status != OK:
        msg = load().she_last_error(handle)
        raise SheError(status, msg.decode() if msg else "")


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def n_shells(n) -> int:
    """Number of radial shells round(|k|) of a grid (the size she_stats fills)."""
    return int(np.floor(np.sqrt(sum(0.25 * v * v for v in n)) + 0.5)) + 1


def current_stream():
    """torch's current HIP stream handle (as an int), or None without a GPU."""
    try:
        import torch
        if torch.cuda.is_available():
            return int(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


@dataclass
class Instance:
    """One realisation (field meanings as in she_instance_desc)."""
    n: tuple = (64,)
    eq: int = HEAT
    bc: int = PERIODIC
    scheme: int = EM
    noise: int = NOISE_INSTANT
    r: float = 0.2
    eps: float = 0.01
    u0: float = 1.0
    u_left: float | None = None
    u_right: float | None = None
    init_sd: float = 0.0
    seed: int = 0
    realisation: int = 0
    cond: object = None      # 1D: N conductivity ratios (material varying along the rod)
    cap: object = None       # 1D: N heat-capacity ratios
    nu: float = 0.0          # BURGERS: Courant number a dt / dx

    @property
    def dim(self) -> int:
        return len(self.n)

    @property
    def ncells(self) -> int:
        return int(np.prod(self.n))

    def c(self) -> InstanceDesc:
        n = tuple(self.n) + (1,) * (3 - len(self.n))
        ul = self.u0 if self.u_left is None else self.u_left
        ur = self.u0 if self.u_right is None else self.u_right
        # the arrays are read during she_create / she_arena_bytes; the caller of
        # c() keeps this object (and so the arrays) alive meanwhile
        self._arrays = [None if a is None else np.ascontiguousarray(a, dtype=np.float64)
                        for a in (self.cond, self.cap)]
        ptrs = [C.POINTER(C.c_double)() if a is None else _dptr(a) for a in self._arrays]
        return InstanceDesc(len(self.n), (C.c_int32 * 3)(*n), self.eq, self.bc, self.scheme, self.noise,
                            self.r, self.eps, self.u0, ul, ur, self.init_sd, self.seed, self.realisation, 0, *ptrs,
                            self.nu)


class Handle:
    """A batch of instances on the GPU (she_create ... she_destroy)."""

    def __init__(self, instances, precision: int = F32, burn_in: int = 0, sample_every: int = 10,
                 stats: int = 0, stream=None, arena=None, block_threads: int = 0, rows_per_block: int = 0,
                 rows_per_group: int = 0, tuning_flags: int = 0, graph_steps: int = 0, tcorr_lags: int = 0,
                 batch_samples: int = 0, flags: int = 0):
        self.lib = load()
        self.instances = list(instances)
        self._descs = (InstanceDesc * len(self.instances))(*[i.c() for i in self.instances])
        if stream is None:
            stream = current_stream()
        self.stream = stream
        self._arena = arena
        cfg = Config(len(self.instances), precision, self._descs, burn_in, sample_every, stats,
                     block_threads, rows_per_block, rows_per_group, tuning_flags, graph_steps, tcorr_lags,
                     batch_samples, flags, C.c_void_p(stream) if stream else None, None, 0)
        if arena is not None:
            cfg.arena = C.c_void_p(arena.data_ptr())
            cfg.arena_bytes = arena.numel() * arena.element_size()
        self._cfg = cfg
        h = C.c_void_p()
        _check(self.lib.she_create(C.byref(cfg), C.byref(h)))
        self.h = h
        self.precision = precision
        self.tcorr_lags = tcorr_lags

    @staticmethod
    def arena_bytes(instances, precision=F32, burn_in=0, sample_every=10, stats=0, block_threads=0,
                    rows_per_block=0, rows_per_group=0, tuning_flags=0, graph_steps=0, tcorr_lags=0,
                    batch_samples=0, flags=0) -> int:
        lib = load()
        insts = list(instances)
        descs = (InstanceDesc * len(insts))(*[i.c() for i in insts])
        cfg = Config(len(insts), precision, descs, burn_in, sample_every, stats, block_threads,
                     rows_per_block, rows_per_group, tuning_flags, graph_steps, tcorr_lags, batch_samples, flags,
                     None, None, 0)
        out = C.c_size_t()
        _check(lib.she_arena_bytes(C.byref(cfg), C.byref(out)))
        return int(out.value)

    @staticmethod
    def tune(instances, precision=F32, stats=0, stream=None, block_threads=0, rows_per_block=0,
             rows_per_group=0, tuning_flags=0, steps: int = 0) -> dict:
        """she_tune: the fastest launch shape for this batch, as keyword
        arguments for Handle (block_threads, rows_per_block, rows_per_group)."""
        lib = load()
        insts = list(instances)
        descs = (InstanceDesc * len(insts))(*[i.c() for i in insts])
        if stream is None:
            stream = current_stream()
        cfg = Config(len(insts), precision, descs, 0, 10, stats, block_threads, rows_per_block, rows_per_group,
                     tuning_flags, 0, 0, 0, 0, C.c_void_p(stream) if stream else None, None, 0)
        out = Config()
        _check(lib.she_tune(C.byref(cfg), int(steps), C.byref(out)))
        return dict(block_threads=int(out.block_threads), rows_per_block=int(out.rows_per_block),
                    rows_per_group=int(out.rows_per_group))

    def close(self):
        if getattr(self, "h", None):
            self.lib.she_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def step(self, nsteps: int):
        _check(self.lib.she_step(self.h, int(nsteps)), self.h)

    def run(self, nsteps: int):
        _check(self.lib.she_run(self.h, int(nsteps)), self.h)

    def reset_stats(self):
        _check(self.lib.she_reset_stats(self.h), self.h)

    @property
    def steps(self) -> int:
        v = C.c_int64()
        _check(self.lib.she_get_step(self.h, C.byref(v)), self.h)
        return int(v.value)

    def read_field(self, i: int) -> np.ndarray:
        n = self.instances[i].ncells
        out = np.zeros(n, dtype=np.float64)
        _check(self.lib.she_read_field(self.h, i, _dptr(out), n), self.h)
        return out

    def write_field(self, i: int, values) -> None:
        v = np.ascontiguousarray(values, dtype=np.float64)
        _check(self.lib.she_write_field(self.h, i, _dptr(v), v.size), self.h)

    def stats(self, i: int, corr: bool = False, sk: bool = False, tcorr: bool = False,
              raise_nonfinite: bool = True, se: bool = False) -> dict:
        inst = self.instances[i]
        n = inst.ncells if inst.dim == 1 else 1
        mean = np.zeros(n)
        var = np.zeros(n)
        out = StatsOut()
        out.mean, out.mean_cap = _dptr(mean), n
        out.var, out.var_cap = _dptr(var), n
        cm = skv = modes = tcv = None
        if tcorr:
            tcv = np.zeros(self.tcorr_lags * n)
            out.tcorr, out.tcorr_cap = _dptr(tcv), tcv.size
        if corr:
            cm = np.zeros(n * n)
            out.corr, out.corr_cap = _dptr(cm), n * n
        if sk:
            nb = inst.ncells if inst.dim == 1 else n_shells(inst.n)
            skv = np.zeros(nb)
            out.sk, out.sk_cap = _dptr(skv), nb
            if inst.dim > 1:
                modes = np.zeros(nb)
                out.sk_modes, out.sk_modes_cap = _dptr(modes), nb
        ses = {}
        if se:
            ses["mean_se"] = np.zeros(n)
            ses["var_se"] = np.zeros(n)
            out.mean_se, out.mean_se_cap = _dptr(ses["mean_se"]), n
            out.var_se, out.var_se_cap = _dptr(ses["var_se"]), n
            if sk:
                ses["sk_se"] = np.zeros(skv.size)
                out.sk_se, out.sk_se_cap = _dptr(ses["sk_se"]), skv.size
        st = self.lib.she_stats(self.h, i, C.byref(out))
        if st != OK and not (st == ENONFINITE and not raise_nonfinite):
            _check(st, self.h)
        res = dict(n_samples=int(out.n_samples), steps=int(out.steps), mean=mean, var=var,
                   sum_u=float(out.sum_u), nonfinite=bool(out.nonfinite), clamp_count=int(out.clamp_count),
                   n_batches=int(out.n_batches), spatial_var=float(out.spatial_var),
                   spatial_var_se=float(out.spatial_var_se))
        res.update(ses)
        if cm is not None:
            res["corr"] = cm.reshape(n, n)
        if skv is not None:
            res["sk"] = skv
        if modes is not None:
            res["sk_modes"] = modes
        if tcv is not None:
            res["tcorr"] = tcv.reshape(self.tcorr_lags, n)
        return res

    def state_bytes(self) -> int:
        v = C.c_size_t()
        _check(self.lib.she_state_bytes(self.h, C.byref(v)), self.h)
        return int(v.value)

    def get_state(self) -> bytes:
        n = self.state_bytes()
        buf = C.create_string_buffer(n)
        _check(self.lib.she_get_state(self.h, buf, n), self.h)
        return buf.raw

    def set_state(self, blob: bytes) -> None:
        buf = C.create_string_buffer(blob, len(blob))
        _check(self.lib.she_set_state(self.h, buf, len(blob)), self.h)


def debug_philox(seed: int, ctr: np.ndarray, stream=None) -> np.ndarray:
    lib = load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    out = np.zeros_like(c)
    _check(lib.she_debug_philox(seed, c.ctypes.data_as(C.POINTER(C.c_uint32)), c.shape[0],
                                out.ctypes.data_as(C.POINTER(C.c_uint32)),
                                C.c_void_p(stream) if stream else None))
    return out


def debug_normals(seed: int, realisation: int, tag: int, step: int, face0: int, count: int,
                  precision: int = F32, stream=None) -> np.ndarray:
    lib = load()
    out = np.zeros(count)
    _check(lib.she_debug_normals(seed, realisation, tag, step, face0, count, precision, _dptr(out),
                                 C.c_void_p(stream) if stream else None))
    return out


def debug_normals_noalloc(seed: int, realisation: int, tag: int, step: int, face0: int, count: int,
                          precision: int = F32, stream=None) -> np.ndarray:
    """she_debug_normals_noalloc: the same numbers, staged in the library's
    fixed per-GPU array (count <= NOALLOC_MAX_NORMALS) instead of an
    allocation."""
    lib = load()
    out = np.zeros(count)
    _check(lib.she_debug_normals_noalloc(seed, realisation, tag, step, face0, count, precision, _dptr(out),
                                         C.c_void_p(stream) if stream else None))
    return out
