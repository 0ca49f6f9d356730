"""Shared test helpers: build oracle descriptions and GPU instances from the
same workload dicts, and run both sides from the same initial field."""
from __future__ import annotations

import numpy as np

import oracle


def f32(v: float) -> float:
    return float(np.float32(v))


def sigma64(inst: dict) -> float:
    return float(np.sqrt(2.0 * inst["r"] * inst["eps"]))


def oracle_desc(inst: dict, precision: int) -> oracle.Desc:
    """FP32 runs feed the oracle the FP32-rounded coefficients the kernels use."""
    r = inst["r"]
    s = sigma64(inst)
    if precision == 0:
        r, s = f32(r), f32(s)
    n = tuple(inst["n"]) + (1,) * (3 - len(inst["n"]))
    return oracle.Desc(dim=len(inst["n"]), n=n, eq=inst["eq"], bc=inst["bc"], scheme=inst["scheme"],
                       noise=inst["noise"], r=r, sigma=s, u0=inst["u0"], u_left=inst["u_left"],
                       u_right=inst["u_right"], init_sd=inst["init_sd"], seed=inst["seed"],
                       realisation=inst["realisation"], cond=inst.get("cond"), cap=inst.get("cap"),
                       nu=f32(inst.get("nu", 0.0)) if precision == 0 else inst.get("nu", 0.0))


def gpu_instance(she, inst: dict):
    return she.Instance(n=tuple(inst["n"]), eq=inst["eq"], bc=inst["bc"], scheme=inst["scheme"],
                        noise=inst["noise"], r=inst["r"], eps=inst["eps"], u0=inst["u0"],
                        u_left=inst["u_left"], u_right=inst["u_right"], init_sd=inst["init_sd"],
                        seed=inst["seed"], realisation=inst["realisation"], cond=inst.get("cond"),
                        cap=inst.get("cap"), nu=inst.get("nu", 0.0))


def max_rel(a: np.ndarray, b: np.ndarray) -> float:
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))
