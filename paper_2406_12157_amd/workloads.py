"""Seeded synthetic workloads (inputs only; no arithmetic of the method).

Each workload is a list of instance parameter dicts with the keys of
``she_instance_desc``: n, eq, bc, scheme, noise, r, eps, u0, u_left, u_right,
init_sd, seed, realisation; plus run parameters (steps, burn_in,
sample_every, precision, stats).  Both the GPU path and the CPU oracle are
driven from these dicts.  The paper measures on no public dataset; these
are synthetic inputs with the shapes and parameter ranges of the benchmark
configurations:

  c1  1D periodic FE, FP64, N = 64, r = 0.2, T0 = 1 uniform, eps = 1e-2
  c2  1D Dirichlet T_L = 1.1, T_R = 0.9, PC, N = 128, FP32 state, r = 0.05,
      eps = 1e-3, linear profile + perturbation, 1e6 steps, full correlation
  c3  2D periodic 512 x 512 x 256 realisations, FE, r = 0.1, eps = 1e-2,
      T0 = 1 + equilibrium perturbation
  c4  1000 1D Dirichlet instances, N log-uniform in [64, 4096], dT/T0 uniform
      in [0, 0.3], FE or PC with probability 1/2 each, r = 0.1, eps = 1e-2
  c5  3D periodic Dean-Kawasaki 256^3, FE, D dt/dx^2 = 0.05, c0 = 1e3 per
      cell volume dV = 1, perturbed start
  burgers  stochastic Burgers ring: N = 256 periodic, c0 = 0.15, r = 0.25,
      Courant number 0.6, eps = 1/dV = 1e-4, perturbed start (batch of
      realisations)
  rod composite rod of the exercises: two materials, the first half with the
      reference properties, the second with conductivity ratio `k_ratio` and
      heat-capacity ratio `c_ratio` (parameters: the paper gives no values
      for the second material), Dirichlet walls, equilibrium or a gradient
"""
from __future__ import annotations

import math

import numpy as np

HEAT, SPECIES, BURGERS = 0, 1, 2
PERIODIC, DIRICHLET = 0, 1
EM, HEUN, BE, CN = 0, 1, 2, 3


def instance(n, eq=HEAT, bc=PERIODIC, scheme=EM, noise=0, r=0.2, eps=1e-2, u0=1.0, u_left=None,
             u_right=None, init_sd=0.0, seed=0, realisation=0, cond=None, cap=None, nu=0.0) -> dict:
    return dict(n=tuple(int(v) for v in n), eq=eq, bc=bc, scheme=scheme, noise=noise, r=float(r),
                eps=float(eps), u0=float(u0), u_left=float(u0 if u_left is None else u_left),
                u_right=float(u0 if u_right is None else u_right), init_sd=float(init_sd), seed=int(seed),
                realisation=int(realisation),
                cond=None if cond is None else tuple(float(v) for v in cond),
                cap=None if cap is None else tuple(float(v) for v in cap), nu=float(nu))


def burgers(n: int = 256, realisations: int = 1, scheme: int = EM, c0: float = 0.15, nu: float = 0.6,
            r: float = 0.25, eps: float = 1e-4, steps: int = 100000) -> dict:
    insts = [instance((n,), eq=BURGERS, scheme=scheme, r=r, eps=eps, u0=c0, nu=nu,
                      init_sd=math.sqrt(eps * c0 * (1 - c0)), realisation=q) for q in range(realisations)]
    return dict(name="burgers_periodic_n%d_x%d" % (n, realisations), precision=0, steps=steps, burn_in=steps // 10,
                sample_every=10, instances=insts)


def rod(n: int = 64, k_ratio: float = 3.0, c_ratio: float = 0.7, t_left: float = 1.1, t_right: float = 0.9,
        scheme: int = EM, r: float = 0.05, eps: float = 1e-3, realisations: int = 1, steps: int = 100000) -> dict:
    """Composite rod: cells [0, n/2) of the reference material, [n/2, n) of
    the second one."""
    cond = [1.0] * (n // 2) + [k_ratio] * (n - n // 2)
    cap = [1.0] * (n // 2) + [c_ratio] * (n - n // 2)
    t0 = 0.5 * (t_left + t_right)
    insts = [instance((n,), bc=DIRICHLET, scheme=scheme, r=r, eps=eps, u0=t0, u_left=t_left, u_right=t_right,
                      init_sd=math.sqrt(eps) * t0, realisation=q, cond=cond, cap=cap) for q in range(realisations)]
    return dict(name="rod_composite_n%d" % n, precision=0, steps=steps, burn_in=steps // 10, sample_every=10,
                instances=insts)


def c1(eps: float = 1e-2) -> dict:
    """The literal eps = 100 (k_B = rho = c_V = 1, dV = 1e-2) is kept as the
    divergence case: c1(eps=100.0)."""
    return dict(name="c1_1d_periodic_fe_fp64_n64", precision=1, steps=100000, burn_in=10000, sample_every=10,
                instances=[instance((64,), r=0.2, eps=eps, u0=1.0, seed=0)])


def c2(realisations: int = 1, steps: int = 1000000) -> dict:
    eps, tl, tr = 1e-3, 1.1, 0.9
    sd = math.sqrt(eps) * 0.5 * (tl + tr)
    return dict(name="c2_1d_dirichlet_pc_n128", precision=0, steps=steps, burn_in=steps // 10, sample_every=10,
                instances=[instance((128,), bc=DIRICHLET, scheme=HEUN, r=0.05, eps=eps, u0=0.5 * (tl + tr),
                                    u_left=tl, u_right=tr, init_sd=sd, seed=0, realisation=q)
                           for q in range(realisations)])


def c3(realisations: int = 256, nx: int = 512, ny: int = 512, steps: int = 10000, scheme: int = EM) -> dict:
    eps = 1e-2
    return dict(name="c3_2d_periodic_%dx%d_x%d" % (nx, ny, realisations), precision=0, steps=steps,
                burn_in=steps // 10, sample_every=10,
                instances=[instance((nx, ny), scheme=scheme, r=0.1, eps=eps, u0=1.0, init_sd=math.sqrt(eps),
                                    seed=0, realisation=q) for q in range(realisations)])


def c4(count: int = 1000, seed: int = 0, n_lo: int = 64, n_hi: int = 4096, steps: int = 10000) -> dict:
    rng = np.random.default_rng(seed)
    u = rng.random(count)
    n = np.rint(n_lo * (n_hi / n_lo) ** u).astype(int)
    dt = 0.3 * rng.random(count)
    scheme = (rng.random(count) < 0.5).astype(int)
    eps = 1e-2
    insts = [instance((int(n[q]),), bc=DIRICHLET, scheme=int(scheme[q]), r=0.1, eps=eps, u0=1.0,
                      u_left=1.0 + 0.5 * dt[q], u_right=1.0 - 0.5 * dt[q], init_sd=0.0, seed=seed, realisation=q)
             for q in range(count)]
    return dict(name="c4_ragged_1d_x%d" % count, precision=0, steps=steps, burn_in=steps // 10, sample_every=10,
                instances=insts)


def c5(n: int = 256, steps: int = 1000) -> dict:
    c0, dv = 1e3, 1.0
    return dict(name="c5_3d_dk_periodic_%d" % n, precision=0, steps=steps, burn_in=steps // 10, sample_every=10,
                instances=[instance((n, n, n), eq=SPECIES, r=0.05, eps=1.0 / dv, u0=c0,
                                    init_sd=math.sqrt(c0 / dv), seed=0)])

