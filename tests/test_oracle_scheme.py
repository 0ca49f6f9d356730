"""Pins for the oracle's deterministic and conservative structure.

* With the noise off, a Fourier mode of the periodic grid is multiplied by
  g_k = 1 - 4 r sum_d sin^2(pi k_d/N_d) per FE step and by (1 + g_k^2)/2 per
  PC step (the discrete amplification factors of the Sec. 3 schemes).
* With noise on, the periodic schemes conserve sum_i U_i (energy / mass,
  Sec. 3 remark on conservation) to round-off.
* With Dirichlet walls the linear profile between the wall values is an exact
  fixed point of the deterministic scheme (ghost stencil T_1 - 3T_0 + 2T_L).
* The Dean-Kawasaki amplitude sqrt(max(n_face, 0)) clamps negative densities.
"""
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("dim,ns,ks", [(1, (32, 1, 1), (3, 0, 0)), (1, (30, 1, 1), (15, 0, 0)),
                                       (2, (16, 12, 1), (2, 5, 0)), (3, (8, 6, 4), (1, 2, 3))])
def test_noise_off_mode_decay(scheme, dim, ns, ks):
    r = 0.11 if dim == 3 else 0.21
    d = oracle.Desc(dim=dim, n=ns, r=r, noise=2, scheme=scheme, u0=1.0)
    grids = np.meshgrid(*[np.arange(n) for n in ns], indexing="ij")
    phase = sum(2 * np.pi * k * (g + 0.5) / n for k, g, n in zip(ks, grids, ns))
    # flatten with x fastest: array index (x, y, z) -> x + nx (y + ny z)
    mode = np.cos(phase).transpose(2, 1, 0).ravel()
    u = 1.0 + 0.1 * mode
    steps = 37
    oracle.advance(d, u, 0, steps)
    x = sum(4 * r * np.sin(np.pi * k / n) ** 2 for k, n in zip(ks, ns))
    g = 1.0 - x
    fac = g if scheme == 0 else 0.5 * (1.0 + g * g)
    np.testing.assert_allclose(u, 1.0 + 0.1 * fac ** steps * mode, rtol=0, atol=1e-13)


@pytest.mark.parametrize("eq", [0, 1])
@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("dim,ns", [(1, (40, 1, 1)), (2, (12, 10, 1)), (3, (6, 4, 8))])
def test_periodic_conservation(eq, scheme, dim, ns):
    u0 = 1.0 if eq == 0 else 50.0
    eps = 0.01 if eq == 0 else 1.0
    r = 0.1
    d = oracle.Desc(dim=dim, n=ns, eq=eq, r=r, sigma=oracle.sigma_of(r, eps), u0=u0,
                    scheme=scheme, init_sd=0.1 * np.sqrt(eps) * u0, seed=5)
    u = oracle.init(d)
    total0 = u.sum()
    oracle.advance(d, u, 0, 400)
    assert np.all(np.isfinite(u))
    assert np.std(u) > 0.01 * np.sqrt(eps * u0 ** 2 if eq == 0 else eps * u0)
    assert abs(u.sum() - total0) <= 1e-12 * abs(total0) * np.sqrt(u.size)


@pytest.mark.parametrize("scheme", [0, 1])
def test_dirichlet_linear_profile_is_fixed_point(scheme):
    N = 24
    d = oracle.Desc(dim=1, n=(N, 1, 1), bc=1, r=0.3, noise=2, scheme=scheme, u_left=0.7, u_right=1.9)
    u = oracle.init(d)
    ref = 0.7 + 1.2 * (np.arange(N) + 0.5) / N
    np.testing.assert_allclose(u, ref, rtol=0, atol=1e-15)
    oracle.advance(d, u, 0, 500)
    np.testing.assert_allclose(u, ref, rtol=0, atol=1e-13)


def test_dirichlet_relaxes_to_profile():
    N = 16
    d = oracle.Desc(dim=1, n=(N, 1, 1), bc=1, r=0.25, noise=2, u_left=1.0, u_right=3.0)
    u = np.full(N, 5.0)
    oracle.advance(d, u, 0, 20000)
    np.testing.assert_allclose(u, 1.0 + 2.0 * (np.arange(N) + 0.5) / N, atol=1e-10)


def test_dirichlet_wall_noise_weight():
    """One FE step from the exact profile with r = 0: the wall faces carry
    sqrt(2) * sigma * T_wall * z, interior faces sigma * T_face * z."""
    N, s = 6, 0.2
    d = oracle.Desc(dim=1, n=(N, 1, 1), bc=1, r=0.0, sigma=s, u_left=2.0, u_right=2.0, seed=1)
    u = np.full(N, 2.0)
    oracle.advance(d, u, 0, 1)
    z = oracle.normals(1, 0, 0, 0, 0, N + 1)
    amp = np.full(N + 1, s * 2.0)
    amp[0] *= np.sqrt(2.0)
    amp[-1] *= np.sqrt(2.0)
    flux = amp * z
    np.testing.assert_allclose(u, 2.0 + flux[1:] - flux[:-1], rtol=0, atol=1e-15)


def test_pc_is_trapezoidal_with_shared_noise():
    """PC = FE predictor, then the average of the old state and an FE step
    from the predictor taken with the same numbers (Sec. 3 PC scheme)."""
    N = 10
    base = dict(dim=1, n=(N, 1, 1), r=0.2, sigma=0.3, u0=1.0, init_sd=0.1, seed=8)
    d_fe = oracle.Desc(scheme=0, **base)
    d_pc = oracle.Desc(scheme=1, **base)
    u = oracle.init(d_fe)
    us = u.copy()
    oracle.advance(d_fe, us, 4, 1)          # predictor
    uss = us.copy()
    oracle.advance(d_fe, uss, 4, 1)         # FE step from the predictor, same step -> same z
    upc = u.copy()
    oracle.advance(d_pc, upc, 4, 1)
    np.testing.assert_allclose(upc, 0.5 * (u + uss), rtol=0, atol=1e-15)


def test_species_clamp_counts_negative_faces():
    N = 8
    d = oracle.Desc(dim=1, n=(N, 1, 1), eq=1, r=0.1, sigma=0.5, u0=1.0, seed=2)
    u = np.array([1.0, -3.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0])
    st = oracle.Stats(d, burn_in=0, every=1000)
    oracle.advance(d, u, 0, 1, st)
    assert st.clamp_count == 2       # faces 1 and 2 have a negative mean density
    z = oracle.normals(2, 0, 0, 0, 0, N)
    u_in = np.array([1.0, -3.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0])
    left = np.roll(u_in, 1)
    face = 0.5 * (left + u_in)
    flux = 0.1 * (u_in - left) + 0.5 * np.sqrt(np.maximum(face, 0)) * z
    np.testing.assert_allclose(u, u_in + np.roll(flux, -1) - flux, atol=1e-15)


def test_literal_large_eps_diverges_and_is_detected():
    """eps = k_B/(rho c_V dV) = 100 at r = 0.2 (k_B = rho = c_V = T0 = 1,
    dV = 1e-2) has an unstable second moment; the oracle flags non-finite."""
    d = oracle.Desc(dim=1, n=(64, 1, 1), r=0.2, sigma=oracle.sigma_of(0.2, 100.0), u0=1.0, seed=0)
    u = oracle.init(d)
    st = oracle.Stats(d, burn_in=0, every=10)
    rc = oracle.advance(d, u, 0, 100000, st)
    assert rc == 1 and st.nonfinite


# ---------------------------------------------------------------- composite rod

HALF = 8
COND = [1.0] * HALF + [3.0] * HALF       # conductivity ratio of the two materials
CAP = [1.0] * HALF + [0.6] * HALF        # heat-capacity ratio


@pytest.mark.parametrize("scheme", [0, 1])
def test_composite_rod_conserves_energy_not_temperature_sum(scheme):
    """Periodic composite rod with noise: sum_i (rho c_V)_i T_i is conserved
    (the scheme is conservative in energy), while sum_i T_i is not."""
    d = oracle.Desc(dim=1, n=(2 * HALF, 1, 1), r=0.08, sigma=0.05, u0=1.0, scheme=scheme, init_sd=0.05, seed=3,
                    cond=COND, cap=CAP)
    u = oracle.init(d)
    e0, s0 = float(np.dot(CAP, u)), float(u.sum())
    oracle.advance(d, u, 0, 2000)
    assert abs(np.dot(CAP, u) - e0) < 1e-12 * abs(e0)
    assert abs(u.sum() - s0) > 1e-4


@pytest.mark.parametrize("scheme", [0, 1])
def test_composite_rod_series_profile_is_fixed_point(scheme):
    """Dirichlet walls with a gradient, noise off: the steady state carries one
    flux J through conductances in series (half cells, walls at a half cell),
    T_i - T_(i-1) = J / g_(i-1/2); it is an exact fixed point, the linear
    profile is not."""
    N, r, tl, tr = 2 * HALF, 0.08, 0.7, 1.3
    lam = np.array(COND)
    g = np.array([lam[0]] + [1.0 / (0.5 / lam[f - 1] + 0.5 / lam[f]) for f in range(1, N)] + [lam[-1]])
    res = np.concatenate([[0.5 / g[0]], 1.0 / g[1:N], [0.5 / g[N]]])   # wall faces: half a cell
    J = (tr - tl) / res.sum()
    prof = tl + J * np.cumsum(res)[:N]
    d = oracle.Desc(dim=1, n=(N, 1, 1), bc=1, r=r, sigma=0.0, u_left=tl, u_right=tr, noise=2, scheme=scheme,
                    cond=COND, cap=CAP)
    u = prof.copy()
    oracle.advance(d, u, 0, 500)
    np.testing.assert_allclose(u, prof, rtol=0, atol=1e-13)
    lin = tl + (tr - tl) * (np.arange(N) + 0.5) / N
    v = lin.copy()
    oracle.advance(d, v, 0, 1)
    assert np.max(np.abs(v - lin)) > 1e-3


def test_composite_rod_with_unit_ratios_is_the_uniform_rod():
    for bc in (0, 1):
        kw = dict(dim=1, n=(12, 1, 1), bc=bc, r=0.2, sigma=0.1, u0=1.0, u_left=0.9, u_right=1.1 if bc else 0.9,
                  init_sd=0.05, seed=7)
        a = oracle.Desc(**kw)
        b = oracle.Desc(**kw, cond=np.ones(12), cap=np.ones(12))
        ua, ub = oracle.init(a), oracle.init(b)
        oracle.advance(a, ua, 0, 300)
        oracle.advance(b, ub, 0, 300)
        np.testing.assert_array_equal(ua, ub)
