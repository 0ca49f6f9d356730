"""FP64 CPU oracle for the stochastic heat / Dean-Kawasaki finite-volume schemes.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library in ``paper_2406_12157_amd`` and never imports it.

The arithmetic lives in ``she_oracle.c`` (plain C, IEEE double,
``-ffp-contract=off``); this module only compiles it with gcc and marshals
arguments through ctypes.  What each C function computes, and which passage of
the paper it follows, is documented in the C file.

Parity status (what pins each part, see the tests under ``tests/``):
  * Philox4x32-10        -- bit-exact against rocRAND's independent engine.
  * Box-Muller normals   -- Kolmogorov-Smirnov and moment tests vs N(0,1).
  * deterministic step   -- Fourier-mode decay by the closed-form amplification
                            factor (FE: 1 - 4 r sum sin^2, PC: (1+g^2)/2).
  * stochastic step      -- conservation to round-off (periodic); exact linear
                            steady profile (Dirichlet); stationary covariance
                            vs discrete Lyapunov solutions and closed forms.
  * statistics           -- estimators checked on hand-made trajectories.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "she_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile she_oracle.c into liboracle.so (gcc, -O2 -ffp-contract=off,
    OpenMP over independent faces and cells)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
             "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Desc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3), ("eq", C.c_int32),
                ("bc", C.c_int32), ("scheme", C.c_int32), ("noise", C.c_int32),
                ("r", C.c_double), ("sigma", C.c_double), ("u0", C.c_double),
                ("u_left", C.c_double), ("u_right", C.c_double),
                ("init_sd", C.c_double), ("seed", C.c_uint64),
                ("realisation", C.c_uint32), ("pad_", C.c_uint32),
                ("face_r", C.POINTER(C.c_double)), ("face_s", C.POINTER(C.c_double)),
                ("cell_w", C.POINTER(C.c_double)), ("nu", C.c_double)]


class _Stats(C.Structure):
    _fields_ = [("burn_in", C.c_int64), ("every", C.c_int64), ("n_samples", C.c_int64),
                ("s1", C.POINTER(C.c_double)), ("s2", C.POINTER(C.c_double)),
                ("m2", C.POINTER(C.c_double)), ("sk", C.POINTER(C.c_double)),
                ("n_bins", C.c_int32), ("pad_", C.c_int32),
                ("sp_mean", C.c_double), ("sp_sq", C.c_double), ("sp_var", C.c_double),
                ("clamp_count", C.c_int64), ("nonfinite", C.c_int32), ("pad2_", C.c_int32),
                ("nonfinite_step", C.c_int64), ("tc_lags", C.c_int64),
                ("tc", C.POINTER(C.c_double)), ("tc_hist", C.POINTER(C.c_double)),
                ("batch_len", C.c_int64), ("batch_cap", C.c_int64),
                ("b_s1", C.POINTER(C.c_double)), ("b_s2", C.POINTER(C.c_double)),
                ("b_sk", C.POINTER(C.c_double)), ("b_sp", C.POINTER(C.c_double))]


def _load():
    global _lib
    if _lib is None:
        build()
        lib = C.CDLL(_LIB)
        lib.or_philox4x32_10.argtypes = [C.POINTER(C.c_uint32)] * 3
        lib.or_normal.restype = C.c_double
        lib.or_normal.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint64]
        lib.or_normals.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64,
                                   C.c_uint64, C.c_int64, C.POINTER(C.c_double)]
        lib.or_ncells.restype = C.c_int64
        lib.or_ncells.argtypes = [C.POINTER(_Desc)]
        lib.or_nfaces.restype = C.c_int64
        lib.or_nfaces.argtypes = [C.POINTER(_Desc)]
        lib.or_n_bins.restype = C.c_int32
        lib.or_n_bins.argtypes = [C.POINTER(_Desc)]
        lib.or_bin_modes.argtypes = [C.POINTER(_Desc), C.POINTER(C.c_double)]
        lib.or_reference.argtypes = [C.POINTER(_Desc), C.POINTER(C.c_double)]
        lib.or_init.restype = C.c_int
        lib.or_init.argtypes = [C.POINTER(_Desc), C.POINTER(C.c_double)]
        lib.or_set_threads.argtypes = [C.c_int]
        lib.or_get_threads.restype = C.c_int
        lib.or_advance.restype = C.c_int
        lib.or_advance.argtypes = [C.POINTER(_Desc), C.POINTER(C.c_double), C.c_int64,
                                   C.c_int64, C.POINTER(_Stats)]
        _lib = lib
    return _lib


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


@dataclass
class Desc:
    """One instance of the scheme (field meanings as in ``she_oracle.c``)."""
    dim: int = 1
    n: tuple = (64, 1, 1)
    eq: int = 0            # 0 heat, 1 Dean-Kawasaki, 2 stochastic Burgers (1D)
    bc: int = 0            # 0 periodic, 1 Dirichlet (1D)
    scheme: int = 0        # 0 FE, 1 PC, 2 backward Euler, 3 Crank-Nicolson (1D)
    noise: int = 0         # 0 instantaneous, 1 deterministic face value, 2 off
    r: float = 0.2
    sigma: float = 0.0
    u0: float = 1.0
    u_left: float = 1.0
    u_right: float = 1.0
    init_sd: float = 0.0
    seed: int = 0
    realisation: int = 0
    cond: object = None    # 1D, optional: N conductivity ratios lambda_i / lambda_ref
    cap: object = None     # 1D, optional: N heat-capacity ratios (rho c_V)_i / (rho c_V)_ref
    nu: float = 0.0        # Burgers: Courant number a dt / dx

    def coefficients(self):
        """Per-face conductance r_f and noise factor s_f, per-cell w_i of a rod
        whose material varies along x (the composite-rod exercise): interior
        faces take the harmonic mean of the two cells' conductivity (series
        resistance of the two half cells), a wall face the adjacent cell's;
        r_f = r lambda_f, s_f = sqrt(2 r_f eps) = sigma sqrt(lambda_f),
        w_i = 1 / cap_i.  None when the rod is uniform."""
        if self.cond is None and self.cap is None:
            return None
        N = int(self.n[0])
        lam = np.ones(N) if self.cond is None else np.asarray(self.cond, dtype=np.float64)
        cap = np.ones(N) if self.cap is None else np.asarray(self.cap, dtype=np.float64)
        nf = N + 1 if self.bc == 1 else N
        lf = np.empty(nf)
        for f in range(nf):
            if self.bc == 1 and f == 0:
                lf[f] = lam[0]
            elif self.bc == 1 and f == N:
                lf[f] = lam[N - 1]
            else:
                a, b = lam[(f - 1) % N], lam[f % N]
                lf[f] = 2.0 * a * b / (a + b)
        return self.r * lf, self.sigma * np.sqrt(lf), 1.0 / cap

    def c(self) -> _Desc:
        n = tuple(self.n) + (1,) * (3 - len(self.n))
        co = self.coefficients()
        null = C.POINTER(C.c_double)()
        if co is not None:
            self._keep = [np.ascontiguousarray(a) for a in co]
        ptrs = [_dptr(a) for a in self._keep] if co is not None else [null, null, null]
        return _Desc(self.dim, (C.c_int32 * 3)(*n), self.eq, self.bc, self.scheme,
                     self.noise, self.r, self.sigma, self.u0, self.u_left, self.u_right,
                     self.init_sd, self.seed, self.realisation, 0, *ptrs, self.nu)

    @property
    def ncells(self) -> int:
        return int(np.prod(self.n))


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (n < 1: every core).  Results
    do not depend on it."""
    _load().or_set_threads(int(n))


def get_threads() -> int:
    return int(_load().or_get_threads())


def philox(ctr, key) -> np.ndarray:
    """Raw Philox4x32-10 block for a 4-word counter and 2-word key."""
    lib = _load()
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib.or_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def normals(seed: int, realisation: int, tag: int, step: int, face0: int, count: int) -> np.ndarray:
    lib = _load()
    out = np.zeros(count, dtype=np.float64)
    lib.or_normals(seed, realisation, tag, step, face0, count, _dptr(out))
    return out


def nfaces(d: Desc) -> int:
    return int(_load().or_nfaces(C.byref(d.c())))


def n_bins(d: Desc) -> int:
    return int(_load().or_n_bins(C.byref(d.c())))


def bin_modes(d: Desc) -> np.ndarray:
    out = np.zeros(n_bins(d), dtype=np.float64)
    _load().or_bin_modes(C.byref(d.c()), _dptr(out))
    return out


def reference(d: Desc) -> np.ndarray:
    out = np.zeros(d.ncells, dtype=np.float64)
    _load().or_reference(C.byref(d.c()), _dptr(out))
    return out


def init(d: Desc) -> np.ndarray:
    out = np.zeros(d.ncells, dtype=np.float64)
    rc = _load().or_init(C.byref(d.c()), _dptr(out))
    if rc != 0:
        raise ValueError("oracle: invalid description (rc=%d)" % rc)
    return out


@dataclass
class Stats:
    """Sample accumulators (FP64) and their finalisation (population moments)."""
    d: Desc
    burn_in: int = 0
    every: int = 1
    per_cell: bool = True
    corr: bool = False
    sk: bool = False
    tcorr_lags: int = 0
    batch: int = 0          # samples per batch of the batch-means error bars (0: none)
    max_batches: int = 0    # batches kept (0: 64)
    _c: _Stats = field(default=None, repr=False)

    def __post_init__(self):
        nc = self.d.ncells
        self.s1 = np.zeros(nc)
        self.s2 = np.zeros(nc)
        self.m2 = np.zeros((nc, nc)) if self.corr else None
        if self.sk:
            self.nb = nc if self.d.dim == 1 else n_bins(self.d)
            self.sk_sum = np.zeros(self.nb)
        else:
            self.nb, self.sk_sum = 0, None
        null = C.POINTER(C.c_double)()
        L = int(self.tcorr_lags)
        if L and self.d.dim != 1:
            raise ValueError("the time correlation is 1D")
        self.tc = np.zeros((L, nc)) if L else None
        self.tc_hist = np.zeros((L, nc)) if L else None
        B = (self.max_batches or 64) if self.batch > 0 else 0
        self.b_s1 = np.zeros((B, nc))
        self.b_s2 = np.zeros((B, nc))
        self.b_sk = np.zeros((B, self.nb))
        self.b_sp = np.zeros((B, 3))
        self._c = _Stats(self.burn_in, self.every, 0,
                         _dptr(self.s1) if self.per_cell else null,
                         _dptr(self.s2) if self.per_cell else null,
                         _dptr(self.m2) if self.corr else null,
                         _dptr(self.sk_sum) if self.sk else null,
                         self.nb, 0, 0.0, 0.0, 0.0, 0, 0, 0, 0, L,
                         _dptr(self.tc) if L else null, _dptr(self.tc_hist) if L else null,
                         int(self.batch), B,
                         _dptr(self.b_s1) if B and self.per_cell else null,
                         _dptr(self.b_s2) if B and self.per_cell else null,
                         _dptr(self.b_sk) if B and self.sk else null,
                         _dptr(self.b_sp) if B else null)

    @property
    def n_samples(self) -> int:
        return int(self._c.n_samples)

    @property
    def nonfinite(self) -> bool:
        return bool(self._c.nonfinite)

    @property
    def clamp_count(self) -> int:
        return int(self._c.clamp_count)

    def mean(self) -> np.ndarray:
        return reference(self.d) + self.s1 / self.n_samples

    def var(self) -> np.ndarray:
        m = self.s1 / self.n_samples
        return self.s2 / self.n_samples - m * m

    def cov(self) -> np.ndarray:
        m = self.s1 / self.n_samples
        return self.m2 / self.n_samples - np.outer(m, m)

    def structure_factor(self) -> np.ndarray:
        """1D: <|T_k|^2> per k.  nD: per radial shell, averaged over its modes."""
        if self.d.dim == 1:
            return self.sk_sum / self.n_samples
        modes = bin_modes(self.d)
        with np.errstate(invalid="ignore", divide="ignore"):
            return self.sk_sum / (self.n_samples * modes)

    def time_corr(self) -> np.ndarray:
        """(L, N): C_i(m) = <d_i(n) d_i(n-m)> - mu_i^2 over the sample pairs
        n >= m (lag m in sampling intervals), mu_i the time mean of d_i;
        NaN where fewer than m + 1 samples were taken."""
        M = self.n_samples
        mu = self.s1 / M
        out = np.full(self.tc.shape, np.nan)
        for m in range(self.tc.shape[0]):
            if M > m:
                out[m] = self.tc[m] / (M - m) - mu * mu
        return out

    def spatial(self):
        """(mean of spatial-mean delta, mean of spatial-mean delta^2, mean spatial variance)."""
        n = self.n_samples
        return self._c.sp_mean / n, self._c.sp_sq / n, self._c.sp_var / n

    # ---- batch means (samples 0..L-1 form batch 0, L..2L-1 batch 1, ...)

    @property
    def n_batches(self) -> int:
        """Complete batches (only the kept ones count)."""
        if self.batch <= 0:
            return 0
        return min(self.n_samples // self.batch, self.b_sp.shape[0])

    def batch_values(self) -> dict:
        """Each statistic formed from the samples of each complete batch alone,
        as the whole-run statistic is formed from all samples: per-cell mean and
        (population) variance, structure factor (1D per k, nD per shell),
        spatial variance.  Arrays with the batch as their first axis."""
        B, L = self.n_batches, float(self.batch)
        m1 = self.b_s1[:B] / L
        out = dict(mean=reference(self.d) + m1, var=self.b_s2[:B] / L - m1 * m1,
                   spatial_var=self.b_sp[:B, 2] / L, spatial_mean=self.b_sp[:B, 0] / L)
        if self.sk:
            if self.d.dim == 1:
                out["sk"] = self.b_sk[:B] / L
            else:
                with np.errstate(invalid="ignore", divide="ignore"):
                    out["sk"] = self.b_sk[:B] / (L * bin_modes(self.d))
        return out

    def se(self) -> dict:
        """Batch-means standard errors: the sample standard deviation of the B
        batch values (divisor B - 1) over sqrt(B); NaN while B < 2."""
        B = self.n_batches
        out = {}
        for k, v in self.batch_values().items():
            if B < 2:
                out[k] = np.full(np.shape(v)[1:], np.nan)
            else:
                out[k] = np.std(v, axis=0, ddof=1) / np.sqrt(B)
        return out


def advance(d: Desc, u: np.ndarray, step0: int, nsteps: int, stats: Stats | None = None) -> int:
    """Advance ``u`` in place; returns 0, or 1 if a sample met a non-finite value."""
    rc = _load().or_advance(C.byref(d.c()), _dptr(u), step0, nsteps,
                            C.byref(stats._c) if stats is not None else None)
    if rc < 0:
        raise ValueError("oracle: invalid description (rc=%d)" % rc)
    return rc


def sigma_of(r: float, eps: float) -> float:
    """Noise factor sqrt(2 r eps) (Sec. 3 discrete noise; Sec. 4 eq. DK with eps = 1/dV)."""
    return float(np.sqrt(2.0 * r * eps))
