"""Pins for the oracle's stochastic Burgers equation (Sec. 5):
dc/dt = -d/dx( a c (1-c) - D dc/dx + sqrt(2 D c (1-c)) Z ), face value the
arithmetic mean, centred hyperbolic flux, FE and PC as for the SHE.

Linearised about a uniform c0 (b = 1 - 2 c0, theta = 2 pi k / N,
x_k = 4 r sin^2(theta/2)), one step maps mode k by
    L_k = -x_k - i nu b sin(theta),   G = 1 + L (FE),   G = 1 + L + L^2/2 (PC),
and the noise of face amplitude sqrt(c0 (1-c0)) enters mode k with variance
N 2 eps c0 (1-c0) x_k, through P = 1 (FE) or P = 1 + L/2 (PC).  The
stationary structure factor of the linearised scheme is then
    S_k = N 2 eps c0 (1-c0) x_k |P|^2 / (1 - |G|^2).
"""
import numpy as np
import pytest

import oracle
from test_oracle_stats import batch_run, mean_se


def desc(**kw):
    base = dict(dim=1, n=(32, 1, 1), eq=2, r=0.25, nu=0.3, u0=0.3, sigma=0.0, seed=5)
    base.update(kw)
    return oracle.Desc(**base)


def linear_factors(N, r, nu, c0, scheme):
    th = 2 * np.pi * np.arange(N) / N
    x = 4 * r * np.sin(th / 2) ** 2
    L = -x - 1j * nu * (1 - 2 * c0) * np.sin(th)
    if scheme == 0:
        return 1 + L, np.ones(N), x
    return 1 + L + 0.5 * L * L, 1 + 0.5 * L, x


@pytest.mark.parametrize("scheme", [0, 1])
def test_burgers_conserves_mass(scheme):
    d = desc(scheme=scheme, sigma=oracle.sigma_of(0.25, 1e-3), init_sd=0.02)
    u = oracle.init(d)
    m0 = u.sum()
    oracle.advance(d, u, 0, 3000)
    assert abs(u.sum() - m0) < 1e-12 * abs(m0)


@pytest.mark.parametrize("scheme", [0, 1])
def test_burgers_particle_hole_symmetry(scheme):
    """c -> 1 - c with a -> -a maps solutions onto solutions (noise off)."""
    rng = np.random.default_rng(3)
    c = 0.3 + 0.2 * rng.random(32)
    a, b = c.copy(), 1.0 - c
    oracle.advance(desc(scheme=scheme, noise=2), a, 0, 200)
    oracle.advance(desc(scheme=scheme, noise=2, nu=-0.3), b, 0, 200)
    np.testing.assert_allclose(a, 1.0 - b, rtol=0, atol=1e-14)


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("k", [1, 3, 7])
def test_burgers_linear_dispersion(scheme, k):
    """A tiny mode on c0 evolves by the complex factor G_k per step: the
    centred hyperbolic flux turns the decay of the diffusive scheme into a
    decaying travelling wave (phase and sign of the advection)."""
    N, r, nu, c0, eps_a = 32, 0.25, 0.3, 0.3, 1e-7
    G, _, _ = linear_factors(N, r, nu, c0, scheme)
    i = np.arange(N)
    c = c0 + eps_a * np.cos(2 * np.pi * k * i / N)
    oracle.advance(desc(scheme=scheme, noise=2), c, 0, 1)
    want = c0 + eps_a * np.real(G[k] * np.exp(2j * np.pi * k * i / N))
    np.testing.assert_allclose(c - c0, want - c0, rtol=0, atol=1e-6 * eps_a)
    # the wave moves: the phase shift is resolved far above the tolerance
    assert abs(np.angle(G[k])) * eps_a > 1e-3 * eps_a


def test_burgers_reduces_to_diffusion_at_half_filling():
    """At c0 = 1/2 the linear advection vanishes (b = 0): S_k is the diffusive
    form N eps c0 (1-c0) / (1 - x_k/2)."""
    G, P, x = linear_factors(32, 0.25, 0.3, 0.5, 0)
    th = 2 * np.pi * np.arange(32) / 32
    k = np.arange(1, 32)
    s_lin = 32 * 2 * 1e-3 * 0.25 * x[k] * np.abs(P[k]) ** 2 / (1 - np.abs(G[k]) ** 2)
    np.testing.assert_allclose(s_lin, 32 * 1e-3 * 0.25 / (1 - x[k] / 2), rtol=1e-12)
    assert np.all(np.abs(np.sin(th[k])) >= 0)


@pytest.mark.parametrize("scheme", [0, 1])
def test_burgers_structure_factor(scheme):
    """Face amplitude at c0, small eps: the measured S_k follows the
    linearised closed form; at b != 0 it differs from the diffusive form."""
    N, r, nu, c0, eps = 32, 0.25, 0.6, 0.15, 1e-4
    d = desc(scheme=scheme, noise=1, sigma=oracle.sigma_of(r, eps), init_sd=np.sqrt(eps * c0 * (1 - c0)),
             seed=91, nu=nu, u0=c0)
    sts = batch_run(d, 20, 20000, 2000, sk=True)
    sk, se = mean_se([s.structure_factor() for s in sts])
    G, P, x = linear_factors(N, r, nu, c0, scheme)
    k = np.arange(1, N)
    want = N * 2 * eps * c0 * (1 - c0) * x[k] * np.abs(P[k]) ** 2 / (1 - np.abs(G[k]) ** 2)
    z = (sk[k] - want) / se[k]
    assert np.max(np.abs(z)) < 4.5, z
    assert np.max(np.abs(sk[k] / want - 1)) < 0.06
    if scheme == 0:   # FE: the centred advection raises S_k well above the diffusive form
        diffusive = N * eps * c0 * (1 - c0) / (1 - x[k] / 2)
        assert np.max(np.abs(want / diffusive - 1)) > 0.4
        assert np.max(np.abs(sk[k] / diffusive - 1)) > 0.4
