"""Closed forms used to pin the oracle's statistics (test-side mathematics).

Derived for the discrete schemes of Sec. 3 of the paper (FE / PC finite-volume
steps with face noise), periodic grids with equal spacing on every axis:

  mode symbol     x_k = 4 r sum_d sin^2(pi k_d / N_d),  FE factor g_k = 1 - x_k
  FE, additive    S_k = N_tot Qbar / (1 - x_k/2)                     (h_k)
  PC, additive    S_k = N_tot Qbar (4 - 2x) / (4 - 2x + x^2)
  per-cell var    Qbar * gamma,  gamma = (1/N_tot) sum_{k != 0} h_k
  SHE, FE, instantaneous face temperature (multiplicative noise):
                  Qbar = eps * m^2 / (1 - eps*beta),
                  beta = (1/N_tot) sum_{k != 0} h_k cos^2(pi k_x / N_x)
  DK, FE          Qbar = m / dV  (the noise variance is linear in n)

Qbar is the mean squared face amplitude: eps * T_face^2 (SHE) or n_face / dV
(DK).  As r -> 0, h_k -> 1 and the per-cell variance tends to
Qbar (1 - 1/N_tot): the paper's equilibrium variance with the periodic
conservation correction (Sec. 3, eq. varcorrT_EQ and the remark after it),
and S_k tends to the flat value of eq. SkTheory (with the cell volume, as the
program evaluates it).

Dirichlet 1D: the scheme is linear in the state when the face amplitude uses
the deterministic profile, so its stationary covariance solves the discrete
Lyapunov equation C = G C G^T + Q; its r -> 0 limit is the continuous
fluctuation-dissipation relation L S + S L^* = B B^* of the supplement.
"""
from __future__ import annotations

import numpy as np


def mode_x(r: float, ns) -> np.ndarray:
    """x_k on the full grid of modes, shape ns (k along each axis 0..N-1)."""
    grids = np.meshgrid(*[np.arange(n) for n in ns], indexing="ij")
    x = np.zeros(tuple(ns))
    for k, n in zip(grids, ns):
        x += 4.0 * r * np.sin(np.pi * k / n) ** 2
    return x


def h_fe(x):
    return 1.0 / (1.0 - 0.5 * x)


def h_pc(x):
    return (4.0 - 2.0 * x) / (4.0 - 2.0 * x + x * x)


def gamma_beta(r: float, ns, scheme: str = "fe"):
    """(gamma, beta_x) sums over k != 0 for a periodic grid."""
    x = mode_x(r, ns)
    h = h_fe(x) if scheme == "fe" else h_pc(x)
    ntot = float(np.prod(ns))
    mask = np.ones(x.shape, dtype=bool)
    mask[(0,) * len(ns)] = False
    kx = np.meshgrid(*[np.arange(n) for n in ns], indexing="ij")[0]
    cos2 = np.cos(np.pi * kx / ns[0]) ** 2
    gamma = float(np.sum(h[mask]) / ntot)
    beta = float(np.sum((h * cos2)[mask]) / ntot)
    return gamma, beta


def qbar_she_fe(eps: float, m: float, r: float, ns) -> float:
    _, beta = gamma_beta(r, ns, "fe")
    return eps * m * m / (1.0 - eps * beta)


def sk_periodic(r: float, ns, qbar: float, scheme: str = "fe") -> np.ndarray:
    x = mode_x(r, ns)
    h = h_fe(x) if scheme == "fe" else h_pc(x)
    return float(np.prod(ns)) * qbar * h


def radial_average(values: np.ndarray, ns) -> tuple[np.ndarray, np.ndarray]:
    """Shell average by round(|k|) with signed k in [-N/2, N/2)."""
    grids = np.meshgrid(*[np.arange(n) for n in ns], indexing="ij")
    k2 = np.zeros(tuple(ns))
    for k, n in zip(grids, ns):
        ks = np.where(2 * k < n, k, k - n)
        k2 += ks.astype(float) ** 2
    bins = np.floor(np.sqrt(k2) + 0.5).astype(int)
    nb = int(np.floor(np.sqrt(sum(0.25 * n * n for n in ns)) + 0.5)) + 1
    sums = np.bincount(bins.ravel(), weights=values.ravel(), minlength=nb)
    cnt = np.bincount(bins.ravel(), minlength=nb).astype(float)
    return sums, cnt


def dirichlet_operators(N: int, r: float, sigma: float, u_left: float, u_right: float,
                        scheme: str = "fe", species: bool = False):
    """Linear one-step map U' = G U + b + B z of the 1D Dirichlet scheme with
    the face amplitude taken from the deterministic (linear) profile."""
    A = np.zeros((N, N))
    for i in range(N):
        A[i, i] = -2.0
        if i > 0:
            A[i, i - 1] = 1.0
        if i < N - 1:
            A[i, i + 1] = 1.0
    A[0, 0] = -3.0
    A[N - 1, N - 1] = -3.0
    G = np.eye(N) + r * A
    # face f = 0..N at x = f dx; deterministic value on the linear profile
    tf = u_left + (u_right - u_left) * np.arange(N + 1) / N
    amp = np.sqrt(np.maximum(tf, 0.0)) if species else tf
    w = np.ones(N + 1)
    w[0] = w[-1] = np.sqrt(2.0)
    D = np.zeros((N, N + 1))
    for i in range(N):
        D[i, i] = -1.0
        D[i, i + 1] = 1.0
    B = D @ np.diag(w * sigma * amp)
    if scheme == "pc":
        I = np.eye(N)
        B = 0.5 * (I + G) @ B
        G = 0.5 * (I + G @ G)
    return G, B


def discrete_lyapunov(G: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Stationary covariance of U' = G U + B z for symmetric G (eigenbasis solve)."""
    lam, V = np.linalg.eigh(0.5 * (G + G.T))
    assert np.allclose(G, G.T, atol=1e-14)
    Q = V.T @ (B @ B.T) @ V
    Ct = Q / (1.0 - np.outer(lam, lam))
    return V @ Ct @ V.T


def composite_operators(r: float, sigma: float, cond, cap, t_left: float, t_right: float,
                        scheme: str = "fe"):
    """One-step map U' = G U + b + B z of a 1D Dirichlet rod whose material
    varies along x, with the face amplitude taken from a uniform temperature
    (equilibrium, t_left == t_right).  Energy balance of cell i:
    (rho c_V)_i dT_i/dt = [J_(i+1/2) - J_(i-1/2)] / dx, with the flux through a
    face driven by the conductance of the two half cells in series, and the
    Dirichlet wall face seeing one half cell.  In units of the reference
    material: conductance g_f / dx^2 * dt, and the noise of a face has
    variance 2 k_B g_f T^2 (fluctuation-dissipation), times sqrt(2) at a wall
    (its ghost-cell half spacing)."""
    assert t_left == t_right, "the amplitude is the equilibrium temperature"
    lam = np.asarray(cond, dtype=float)
    cap = np.asarray(cap, dtype=float)
    N = lam.size
    # series conductance of faces 0..N: two half cells (interior), one half cell and the wall
    g = np.empty(N + 1)
    g[0], g[N] = lam[0], lam[N - 1]
    for f in range(1, N):
        g[f] = 1.0 / (0.5 / lam[f - 1] + 0.5 / lam[f])
    A = np.zeros((N, N))
    for i in range(N):
        lo, hi = (2.0 * g[0] if i == 0 else g[i]), (2.0 * g[N] if i == N - 1 else g[i + 1])
        A[i, i] = -(lo + hi)
        if i > 0:
            A[i, i - 1] = g[i]
        if i < N - 1:
            A[i, i + 1] = g[i + 1]
    Winv = np.diag(1.0 / cap)
    G = np.eye(N) + r * Winv @ A
    wall = np.ones(N + 1)
    wall[0] = wall[-1] = np.sqrt(2.0)
    D = np.zeros((N, N + 1))
    for i in range(N):
        D[i, i], D[i, i + 1] = -1.0, 1.0
    B = Winv @ D @ np.diag(wall * sigma * np.sqrt(g) * t_left)
    if scheme == "pc":
        I = np.eye(N)
        B = 0.5 * (I + G) @ B
        G = 0.5 * (I + G @ G)
    return G, B


def general_discrete_lyapunov(G: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Stationary covariance C = G C G^T + B B^T for any stable G."""
    from scipy.linalg import solve_discrete_lyapunov
    return solve_discrete_lyapunov(G, B @ B.T)


def garcia_neq_correlation(N: int, eps_dv: float, t_mean: np.ndarray, grad_t: float,
                           ell: float = 1.0, area_eps: float | None = None) -> np.ndarray:
    """Paper's eq. TcorrNEQ in units where the length is ell and
    k_B/(rho c_V dV) = eps_dv, so k_B/(rho c_V A ell) = eps_dv * dx / ell."""
    dx = ell / N
    x = (np.arange(N) + 0.5) * dx
    diag = eps_dv * t_mean ** 2
    pref = eps_dv * dx * grad_t ** 2 / ell
    xi, xj = np.meshgrid(x, x, indexing="ij")
    lr = np.where(xi < xj, xi * (ell - xj), xj * (ell - xi))
    return np.diag(diag) + pref * lr
