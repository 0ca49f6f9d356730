"""Pins for the oracle's implicit schemes (the implicit-scheme exercise):
diffusion at theta = 1 (backward Euler) or 1/2 (Crank-Nicolson), noise
explicit with the face amplitude of U^n:
    (I - theta W A) U' = U + (1 - theta) W (A U + b) + theta W b + noise.

Periodic mode k (x_k = 4 r sin^2(pi k/N)): one step maps it by
    G_k = (1 - (1 - theta) x_k) / (1 + theta x_k),
and the additive noise of variance 2 eps Q x_k (per mode, times N) enters
through 1 / (1 + theta x_k), so the stationary structure factor is
    S_k = N eps Q / (1 + x_k/2)   (backward Euler),
    S_k = N eps Q                 (Crank-Nicolson: flat for every r).
"""
import numpy as np
import pytest

import oracle
import theory
from test_oracle_stats import batch_run, mean_se

BE, CN = 2, 3


def mode_factor(x, scheme):
    th = 1.0 if scheme == BE else 0.5
    return (1 - (1 - th) * x) / (1 + th * x)


@pytest.mark.parametrize("scheme", [BE, CN])
@pytest.mark.parametrize("k", [1, 5, 8])
def test_implicit_mode_decay_beyond_the_explicit_limit(scheme, k):
    N, r = 16, 3.0                       # six times the explicit stability limit
    d = oracle.Desc(dim=1, n=(N, 1, 1), r=r, sigma=0.0, u0=1.0, noise=2, scheme=scheme)
    i = np.arange(N)
    mode = np.cos(2 * np.pi * k * (i + 0.5) / N)
    u = 1.0 + 0.1 * mode
    steps = 7
    oracle.advance(d, u, 0, steps)
    x = 4 * r * np.sin(np.pi * k / N) ** 2
    np.testing.assert_allclose(u, 1.0 + 0.1 * mode_factor(x, scheme) ** steps * mode, rtol=0, atol=1e-13)


@pytest.mark.parametrize("scheme", [BE, CN])
def test_implicit_dirichlet_profile_and_conservation(scheme):
    N = 12
    lin = 0.8 + 0.4 * (np.arange(N) + 0.5) / N
    d = oracle.Desc(dim=1, n=(N, 1, 1), bc=1, r=2.5, sigma=0.0, u_left=0.8, u_right=1.2, noise=2, scheme=scheme)
    u = lin.copy()
    oracle.advance(d, u, 0, 50)
    np.testing.assert_allclose(u, lin, rtol=0, atol=1e-13)
    # periodic, with (multiplicative) noise: the sum is conserved
    p = oracle.Desc(dim=1, n=(N, 1, 1), r=2.5, sigma=0.05, u0=1.0, scheme=scheme, init_sd=0.05, seed=4)
    v = oracle.init(p)
    s0 = v.sum()
    oracle.advance(p, v, 0, 500)
    assert abs(v.sum() - s0) < 1e-12 * s0


@pytest.mark.parametrize("scheme", [BE, CN])
def test_implicit_structure_factor(scheme):
    """Additive noise (face amplitude at u0), r = 2: BE damps S_k by
    1/(1 + x_k/2); Crank-Nicolson keeps it flat at N eps u0^2."""
    N, r, eps, m = 16, 2.0, 0.01, 1.0
    d = oracle.Desc(dim=1, n=(N, 1, 1), r=r, sigma=oracle.sigma_of(r, eps), u0=m, noise=1, scheme=scheme,
                    init_sd=np.sqrt(eps), seed=23)
    sts = batch_run(d, 20, 10000, 500, sk=True)
    sk, se = mean_se([s.structure_factor() for s in sts])
    x = theory.mode_x(r, (N,))
    k = np.arange(1, N)
    flat = N * eps * m * m
    want = flat / (1 + x[k] / 2) if scheme == BE else np.full(N - 1, flat)
    assert np.max(np.abs((sk[k] - want) / se[k])) < 4.5
    assert np.max(np.abs(sk[k] / want - 1)) < 0.08
    if scheme == BE:
        assert sk[N // 2] < 0.4 * flat                 # x = 8 at k = N/2: S_k = flat / 5


@pytest.mark.parametrize("scheme", [BE, CN])
def test_implicit_dirichlet_covariance_vs_lyapunov(scheme):
    """Dirichlet walls with a gradient, face amplitude on the linear profile,
    r = 1.5: the covariance equals the discrete Lyapunov solution of
    U' = G U + B z, G = M^-1 (I + (1 - theta) r A), B = M^-1 D S,
    M = I - theta r A."""
    N, r, eps, tl, tr = 8, 1.5, 0.01, 0.5, 1.5
    sigma = oracle.sigma_of(r, eps)
    d = oracle.Desc(dim=1, n=(N, 1, 1), bc=1, r=r, sigma=sigma, u_left=tl, u_right=tr, noise=1, scheme=scheme,
                    seed=57)
    sts = batch_run(d, 20, 20000, 500, corr=True)
    C, se = mean_se([s.cov() for s in sts])
    th = 1.0 if scheme == BE else 0.5
    G1, B1 = theory.dirichlet_operators(N, r, sigma, tl, tr, "fe")    # G1 = I + r A, B1 = D S
    A = (G1 - np.eye(N)) / r
    M = np.eye(N) - th * r * A
    G = np.linalg.solve(M, np.eye(N) + (1 - th) * r * A)
    B = np.linalg.solve(M, B1)
    want = theory.general_discrete_lyapunov(G, B)
    assert np.max(np.abs((C - want) / se)) < 5.0
    np.testing.assert_allclose(np.diag(C), np.diag(want), rtol=0.05)
