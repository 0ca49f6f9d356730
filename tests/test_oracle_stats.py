"""Statistical pins for the oracle: stationary covariances and structure
factors of the discrete schemes against closed forms and Lyapunov solutions
(``tests/theory.py``), with batch-means error bars, plus the estimators
themselves against numpy on recorded trajectories.
"""
import numpy as np
import pytest

import oracle
import theory


def batch_run(d, nbatch, steps_per_batch, relax, every=1, **kw):
    """Equilibrate, then run nbatch consecutive batches with fresh
    accumulators; returns the list of Stats."""
    u = oracle.init(d)
    batch_run.mean0 = u.mean()      # conserved under periodic walls
    oracle.advance(d, u, 0, relax)
    out, t = [], relax
    for _ in range(nbatch):
        st = oracle.Stats(d, burn_in=0, every=every, **kw)
        assert oracle.advance(d, u, t, steps_per_batch, st) == 0
        t += steps_per_batch
        out.append(st)
    return out


def mean_se(values):
    v = np.asarray(values)
    return v.mean(axis=0), v.std(axis=0, ddof=1) / np.sqrt(v.shape[0])


def test_estimators_match_numpy_on_a_recorded_trajectory():
    N = 12
    d = oracle.Desc(dim=1, n=(N, 1, 1), r=0.2, sigma=0.3, u0=1.0, init_sd=0.2, seed=4)
    u = oracle.init(d)
    st = oracle.Stats(d, burn_in=3, every=2, corr=True, sk=True)
    traj = []
    for t in range(40):
        oracle.advance(d, u, t, 1, st)
        if t + 1 > 3 and (t + 1) % 2 == 0:
            traj.append(u.copy())
    X = np.array(traj)
    assert st.n_samples == len(traj)
    np.testing.assert_allclose(st.mean(), X.mean(0), atol=1e-13)
    np.testing.assert_allclose(st.var(), X.var(0), atol=1e-13)
    np.testing.assert_allclose(st.cov(), np.cov(X.T, bias=True), atol=1e-13)
    sk = (np.abs(np.fft.fft(X, axis=1)) ** 2).mean(0)
    np.testing.assert_allclose(st.structure_factor(), sk, rtol=1e-12)
    sp = st.spatial()
    dl = X - 1.0
    np.testing.assert_allclose(sp[2], (dl.var(axis=1)).mean(), atol=1e-14)


def test_radial_structure_factor_matches_numpy_fft2():
    ns = (8, 6)
    d = oracle.Desc(dim=2, n=ns + (1,), r=0.1, sigma=0.2, u0=1.0, init_sd=0.3, seed=6)
    u = oracle.init(d)
    st = oracle.Stats(d, burn_in=0, every=1, sk=True)
    acc = np.zeros(ns)
    for t in range(6):
        oracle.advance(d, u, t, 1, st)
        field = u.reshape(ns[1], ns[0]).T        # index (x, y)
        acc += np.abs(np.fft.fft2(field)) ** 2
    sums, cnt = theory.radial_average(acc / 6, ns)
    with np.errstate(invalid="ignore"):
        want = sums / cnt
    got = st.structure_factor()
    ok = cnt > 0
    np.testing.assert_allclose(got[ok], want[ok], rtol=1e-12)
    np.testing.assert_array_equal(oracle.bin_modes(d), cnt)


@pytest.mark.parametrize("scheme", ["fe", "pc"])
def test_additive_periodic_structure_factor(scheme):
    """Deterministic face temperature: S_k = N eps m^2 h_k exactly."""
    N, r, eps, m = 16, 0.2, 0.01, 1.0
    d = oracle.Desc(dim=1, n=(N, 1, 1), r=r, sigma=oracle.sigma_of(r, eps), u0=m, noise=1,
                    scheme=0 if scheme == "fe" else 1, init_sd=np.sqrt(eps) * m, seed=21)
    sts = batch_run(d, 20, 20000, 2000, sk=True)
    sk, se = mean_se([s.structure_factor() for s in sts])
    want = theory.sk_periodic(r, (N,), eps * m * m, scheme)
    k = np.arange(1, N)
    z = (sk[k] - want[k]) / se[k]
    assert np.max(np.abs(z)) < 4.5, z
    assert np.max(np.abs(sk[k] / want[k] - 1)) < 0.08
    # the r -> 0 flat value of eq. SkTheory is off by h_k (up to 1.67 for FE)
    if scheme == "fe":
        assert sk[N // 2] / (N * eps * m * m) > 1.5


def test_multiplicative_fe_variance_closed_form():
    """Instantaneous face temperature, FE, periodic: per-cell variance
    eps m^2 gamma / (1 - eps beta)."""
    N, r, eps, m = 16, 0.2, 0.1, 1.0
    d = oracle.Desc(dim=1, n=(N, 1, 1), r=r, sigma=oracle.sigma_of(r, eps), u0=m,
                    init_sd=np.sqrt(eps) * m, seed=31)
    sts = batch_run(d, 20, 25000, 2000)
    m = batch_run.mean0
    v, se = mean_se([s.var().mean() for s in sts])
    gamma, beta = theory.gamma_beta(r, (N,))
    want = eps * m * m * gamma / (1 - eps * beta)
    linear = eps * m * m * gamma
    assert abs(v - want) < 4.5 * se, (v, want, se)
    assert abs(want - linear) > 6 * se     # the nonlinear correction is resolved


def test_species_fe_structure_factor():
    """Dean-Kawasaki FE periodic: S_k = N (m/dV) h_k (noise variance linear in n)."""
    N, r, dv, m = 16, 0.2, 1.0, 200.0
    eps = 1.0 / dv
    d = oracle.Desc(dim=1, n=(N, 1, 1), eq=1, r=r, sigma=oracle.sigma_of(r, eps), u0=m,
                    init_sd=np.sqrt(m / dv), seed=41)
    sts = batch_run(d, 20, 20000, 2000, sk=True)
    m = batch_run.mean0
    sk, se = mean_se([s.structure_factor() for s in sts])
    want = theory.sk_periodic(r, (N,), m / dv, "fe")
    k = np.arange(1, N)
    assert np.max(np.abs((sk[k] - want[k]) / se[k])) < 4.5
    assert sum(s.clamp_count for s in sts) == 0


@pytest.mark.parametrize("scheme", ["fe", "pc"])
def test_dirichlet_covariance_vs_discrete_lyapunov(scheme):
    """Deterministic face temperature, Dirichlet walls with a gradient: the
    full covariance equals the discrete Lyapunov solution."""
    N, r, eps, tl, tr = 8, 0.2, 0.01, 0.5, 1.5
    sigma = oracle.sigma_of(r, eps)
    d = oracle.Desc(dim=1, n=(N, 1, 1), bc=1, r=r, sigma=sigma, u_left=tl, u_right=tr, noise=1,
                    scheme=0 if scheme == "fe" else 1, seed=51)
    sts = batch_run(d, 20, 20000, 1000, corr=True)
    C, se = mean_se([s.cov() for s in sts])
    G, B = theory.dirichlet_operators(N, r, sigma, tl, tr, scheme)
    want = theory.discrete_lyapunov(G, B)
    z = (C - want) / se
    assert np.max(np.abs(z)) < 5.0, np.max(np.abs(z))
    np.testing.assert_allclose(np.diag(C), np.diag(want), rtol=0.05)
    # the mean is the linear profile
    mean = np.mean([s.mean() for s in sts], axis=0)
    np.testing.assert_allclose(mean, tl + (tr - tl) * (np.arange(N) + 0.5) / N, atol=5e-3)


def test_dirichlet_equilibrium_matches_paper_in_small_r_limit():
    """At small r the Dirichlet equilibrium covariance approaches the paper's
    eq. varcorrT_EQ (eps T^2 on the diagonal, zero elsewhere), which the
    sqrt(2) wall noise makes exact in the semi-discrete limit."""
    N, r, eps, t0 = 8, 0.02, 0.01, 1.0
    sigma = oracle.sigma_of(r, eps)
    G, B = theory.dirichlet_operators(N, r, sigma, t0, t0, "pc")
    want = theory.discrete_lyapunov(G, B)
    np.testing.assert_allclose(want, eps * t0 ** 2 * np.eye(N), atol=2e-3 * eps)
    d = oracle.Desc(dim=1, n=(N, 1, 1), bc=1, r=r, sigma=sigma, u_left=t0, u_right=t0,
                    scheme=1, init_sd=np.sqrt(eps) * t0, seed=61)
    sts = batch_run(d, 20, 30000, 5000, every=5)
    v, se = mean_se([s.var() for s in sts])
    assert np.max(np.abs(v - eps * t0 ** 2) / se) < 4.5


def test_2d_fe_spatial_variance_and_radial_sk():
    ns, r, eps, m = (8, 8), 0.1, 0.01, 1.0
    d = oracle.Desc(dim=2, n=ns + (1,), r=r, sigma=oracle.sigma_of(r, eps), u0=m, noise=1,
                    init_sd=np.sqrt(eps) * m, seed=71)
    sts = batch_run(d, 16, 6000, 1000, every=2, sk=True)
    sp, se = mean_se([s.spatial()[2] for s in sts])
    gamma, _ = theory.gamma_beta(r, ns)
    want = eps * m * m * gamma
    assert abs(sp - want) < 4.5 * se
    sk, sk_se = mean_se([s.structure_factor() for s in sts])
    sums, cnt = theory.radial_average(theory.sk_periodic(r, ns, eps * m * m), ns)
    ok = cnt > 0
    ok[0] = False
    wantk = sums[ok] / cnt[ok]
    assert np.max(np.abs((sk[ok] - wantk) / sk_se[ok])) < 4.5


def test_3d_species_variance():
    ns, r, dv, m = (6, 6, 6), 0.05, 1.0, 100.0
    d = oracle.Desc(dim=3, n=ns, eq=1, r=r, sigma=oracle.sigma_of(r, 1.0 / dv), u0=m,
                    init_sd=np.sqrt(m / dv), seed=81)
    sts = batch_run(d, 16, 2500, 500, every=2)
    m = batch_run.mean0
    sp, se = mean_se([s.spatial()[2] for s in sts])
    gamma, _ = theory.gamma_beta(r, ns)
    assert abs(sp - m / dv * gamma) < 4.5 * se


def test_garcia_long_range_correlation_is_the_scheme_limit():
    """The paper's eq. TcorrNEQ equals, off the diagonal, the r -> 0 limit of
    the discrete Dirichlet covariance (continuous Lyapunov equation of the
    supplement for the semi-discrete system), for a 1:5 wall ratio."""
    import scipy.linalg as sla
    N, eps, tl, tr = 32, 1e-3, 1.0, 5.0
    # semi-discrete: dU = (A/dx^2) U dt + noise; in units dt' = kappa t/dx^2
    G, B = theory.dirichlet_operators(N, 1.0, np.sqrt(2 * eps), tl, tr, "fe")
    L = G - np.eye(N)                          # = A (r = 1)
    S = sla.solve_continuous_lyapunov(L, -B @ B.T)
    tbar = tl + (tr - tl) * (np.arange(N) + 0.5) / N
    want = theory.garcia_neq_correlation(N, eps, tbar, tr - tl)
    off = ~np.eye(N, dtype=bool)
    amp = np.max(np.abs(want[off]))
    # the column the paper plots (x_j = l/4), off the diagonal
    j = N // 4
    col = np.arange(N) != j
    assert np.max(np.abs(S[col, j] - want[col, j])) < 0.01 * amp
    # away from the diagonal everywhere; next to it the face-to-face change of
    # the multiplicative amplitude adds an O(eps dT T / N) term the theory omits
    far = np.abs(np.subtract.outer(np.arange(N), np.arange(N))) >= 4
    assert np.max(np.abs(S[far] - want[far])) < 0.05 * amp
    np.testing.assert_allclose(np.diag(S), np.diag(want), rtol=0.05)


# ---------------------------------------------------------------- time correlation

def test_time_correlation_estimator_matches_numpy():
    N = 12
    d = oracle.Desc(dim=1, n=(N, 1, 1), r=0.2, sigma=0.3, u0=1.0, init_sd=0.2, seed=4)
    u = oracle.init(d)
    st = oracle.Stats(d, burn_in=3, every=2, tcorr_lags=6)
    traj = []
    for t in range(60):
        oracle.advance(d, u, t, 1, st)
        if t + 1 > 3 and (t + 1) % 2 == 0:
            traj.append(u.copy() - 1.0)
    X = np.array(traj)
    mu = X.mean(0)
    got = st.time_corr()
    for m in range(6):
        want = (X[m:] * X[:len(X) - m]).mean(0) - mu * mu
        np.testing.assert_allclose(got[m], want, atol=1e-14)


@pytest.mark.parametrize("scheme", [0, 1])
def test_time_correlation_of_a_decaying_mode(scheme):
    """Noise off, one Fourier mode a cos(2 pi k (i+1/2)/N): the state after t
    steps is the mode times G^t (G = g for FE, (1+g^2)/2 for PC, g = 1 - x_k),
    so the lag sums are geometric series in closed form."""
    N, r, k0, a, every, burn = 16, 0.15, 3, 0.4, 3, 7
    d = oracle.Desc(dim=1, n=(N, 1, 1), r=r, sigma=0.0, u0=2.0, noise=2, scheme=scheme, seed=1)
    c = np.cos(2 * np.pi * k0 * (np.arange(N) + 0.5) / N)
    u = 2.0 + a * c
    L, steps = 9, 200
    st = oracle.Stats(d, burn_in=burn, every=every, tcorr_lags=L)
    oracle.advance(d, u, 0, steps, st)
    g = 1 - 4 * r * np.sin(np.pi * k0 / N) ** 2
    G = g if scheme == 0 else 0.5 * (1 + g * g)
    t_first = (burn // every + 1) * every          # first sample step
    M = st.n_samples
    assert M == (steps - t_first) // every + 1
    for m in range(L):
        # sum_{n=m}^{M-1} G^(t_n + t_(n-m)), t_n = t_first + n every
        geo = sum(G ** (2 * t_first + (2 * n - m) * every) for n in range(m, M))
        np.testing.assert_allclose(st.tc[m], a * a * c * c * geo, rtol=1e-10, atol=1e-300)


@pytest.mark.parametrize("case", ["fe_instantaneous", "pc_frozen"])
def test_time_correlation_closed_form(case):
    """Periodic stationary state: <dU_i^(n+m) dU_i^n> = (1/N^2) sum_{k != 0}
    G_k^m S_k.  The lag-m map of mode k is G_k^m and the noise of later steps
    is uncorrelated with the earlier state (exact for FE also with the
    state-dependent face amplitude, and for additive PC)."""
    N, r, L = 16, 0.2, 24
    if case == "fe_instantaneous":
        eps, noise, scheme = 0.1, 0, 0
    else:
        eps, noise, scheme = 0.01, 1, 1
    d = oracle.Desc(dim=1, n=(N, 1, 1), r=r, sigma=oracle.sigma_of(r, eps), u0=1.0, noise=noise,
                    scheme=scheme, init_sd=np.sqrt(eps), seed=51)
    sts = batch_run(d, 20, 20000, 2000, tcorr_lags=L)
    m0 = batch_run.mean0
    tc, se = mean_se([s.time_corr().mean(axis=1) for s in sts])
    x = theory.mode_x(r, (N,))
    g = 1 - x
    if scheme == 0:
        G, sk = g, theory.sk_periodic(r, (N,), theory.qbar_she_fe(eps, m0, r, (N,)), "fe")
    else:
        G, sk = 0.5 * (1 + g * g), theory.sk_periodic(r, (N,), eps * 1.0, "pc")
    k = np.arange(1, N)
    want = np.array([np.sum(G[k] ** m * sk[k]) / N ** 2 for m in range(L)])
    z = (tc - want) / se
    assert np.max(np.abs(z)) < 4.5, z
    assert np.max(np.abs(tc[:8] / want[:8] - 1)) < 0.05
    # the correlation decays: lag 23 keeps well under half of lag 0
    assert want[L - 1] < 0.5 * want[0]


@pytest.mark.parametrize("scheme", ["fe", "pc"])
def test_composite_rod_equilibrium_covariance(scheme):
    """Iron-like / aluminium-like halves (conductivity ratio 3, heat-capacity
    ratio 0.6), Dirichlet walls at the same temperature, face amplitude at that
    temperature: the full covariance is the discrete Lyapunov solution of the
    composite scheme's linear map."""
    N, r, eps, t0 = 8, 0.05, 0.01, 1.0
    cond, cap = [1.0] * 4 + [3.0] * 4, [1.0] * 4 + [0.6] * 4
    sigma = oracle.sigma_of(r, eps)
    d = oracle.Desc(dim=1, n=(N, 1, 1), bc=1, r=r, sigma=sigma, u_left=t0, u_right=t0, noise=1,
                    scheme=0 if scheme == "fe" else 1, init_sd=np.sqrt(eps), seed=71, cond=cond, cap=cap)
    sts = batch_run(d, 20, 20000, 2000, corr=True)
    C, se = mean_se([s.cov() for s in sts])
    G, B = theory.composite_operators(r, sigma, cond, cap, t0, t0, scheme)
    want = theory.general_discrete_lyapunov(G, B)
    assert np.max(np.abs((C - want) / se)) < 5.0
    np.testing.assert_allclose(np.diag(C), np.diag(want), rtol=0.05)


def test_composite_rod_equilibrium_variance_follows_heat_capacity():
    """Exercise on the composite rod at equilibrium: the fluctuation-
    dissipation balance gives <dT_i^2> = eps T^2 / cap_i, set by the local
    heat capacity and not by the conductivity; the cross-correlations vanish.
    Exact for the semi-discrete scheme (the continuous Lyapunov equation),
    approached by the discrete schemes as r -> 0."""
    N, eps, t0 = 8, 0.01, 1.0
    cond, cap = [1.0] * 4 + [3.0] * 4, [1.0] * 4 + [0.6] * 4
    sigma0 = oracle.sigma_of(1.0, eps)
    # semi-discrete: (W A) C + C (W A)^T + B B^T = 0 at unit rate solves to eps T^2 W^-1
    from scipy.linalg import solve_continuous_lyapunov
    G, B = theory.composite_operators(1.0, sigma0, cond, cap, t0, t0, "fe")
    cont = solve_continuous_lyapunov(G - np.eye(N), -B @ B.T)
    np.testing.assert_allclose(cont, eps * t0 ** 2 * np.diag(1.0 / np.array(cap)), atol=1e-15)
    # the discrete schemes approach it as r -> 0: error O(r) for FE, O(r^2) for PC
    limit = eps * t0 ** 2 * np.diag(1.0 / np.array(cap))
    for scheme, order in (("fe", 1), ("pc", 2)):
        err = []
        for r in (0.02, 0.01, 0.005):
            G, B = theory.composite_operators(r, oracle.sigma_of(r, eps), cond, cap, t0, t0, scheme)
            err.append(np.max(np.abs(theory.general_discrete_lyapunov(G, B) - limit)) / eps)
        for a, b in zip(err, err[1:]):
            assert 0.8 * 2 ** order < a / b < 1.25 * 2 ** order, (scheme, err)
    # the oracle at r = 0.02 (PC, face amplitude at the equilibrium temperature)
    r = 0.02
    sigma = oracle.sigma_of(r, eps)
    d = oracle.Desc(dim=1, n=(N, 1, 1), bc=1, r=r, sigma=sigma, u_left=t0, u_right=t0, scheme=1, noise=1,
                    init_sd=np.sqrt(eps), seed=81, cond=cond, cap=cap)
    sts = batch_run(d, 20, 30000, 5000, every=5)
    v, se = mean_se([s.var() for s in sts])
    G, B = theory.composite_operators(r, sigma, cond, cap, t0, t0, "pc")
    want = np.diag(theory.general_discrete_lyapunov(G, B))
    assert np.max(np.abs(v - want) / se) < 4.5, (v, want, se)
    assert v[6] / v[1] > 1.4          # the low-capacity half fluctuates more


# ---------------------------------------------------------------- batch-means error bars

@pytest.mark.parametrize("dim", [1, 2])
def test_batch_means_match_numpy_on_a_recorded_trajectory(dim):
    """The oracle's per-batch statistics and standard errors against numpy on
    the recorded samples of the same run: the samples reshaped into B
    consecutive batches of L, each statistic formed per batch (per-cell mean
    and population variance, |DFT|^2 per k or shell average, spatial
    variance), SE = std over batches (ddof 1) / sqrt(B); the samples of an
    incomplete last batch enter the totals only."""
    if dim == 1:
        d = oracle.Desc(dim=1, n=(12, 1, 1), bc=1, scheme=1, r=0.2, sigma=0.3, u0=1.0, u_left=1.2, u_right=0.9,
                        init_sd=0.2, seed=4)
    else:
        d = oracle.Desc(dim=2, n=(8, 6, 1), r=0.1, sigma=0.2, u0=1.0, init_sd=0.3, seed=6)
    L, every, burn = 7, 2, 5
    u = oracle.init(d)
    st = oracle.Stats(d, burn_in=burn, every=every, sk=True, batch=L)
    ref = oracle.reference(d)
    traj = []
    for t in range(2 * (burn + 3 * L + 4 * L + 3)):
        oracle.advance(d, u, t, 1, st)
        if t + 1 > burn and (t + 1) % every == 0:
            traj.append(u.copy())
    X = np.array(traj)
    M = len(traj)
    B = M // L
    assert st.n_samples == M and st.n_batches == B >= 6 and M % L != 0
    Xb = X[:B * L].reshape(B, L, -1)
    D = Xb - ref
    bv = st.batch_values()
    np.testing.assert_allclose(bv["mean"], Xb.mean(axis=1), rtol=1e-13)
    np.testing.assert_allclose(bv["var"], D.var(axis=1), atol=1e-14)
    np.testing.assert_allclose(bv["spatial_var"], D.var(axis=2).mean(axis=1), atol=1e-14)
    if dim == 1:
        skb = (np.abs(np.fft.fft(Xb, axis=2)) ** 2).mean(axis=1)
    else:
        p = (np.abs(np.fft.fft2(Xb.reshape(B, L, d.n[1], d.n[0]))) ** 2).mean(axis=1)   # [B][ky][kx]
        modes = theory.radial_average(np.ones((d.n[0], d.n[1])), (d.n[0], d.n[1]))[1]
        ok = modes > 0
        skb = np.array([theory.radial_average(p[b].T, (d.n[0], d.n[1]))[0][ok] / modes[ok] for b in range(B)])
        bv["sk"] = bv["sk"][:, ok]
    np.testing.assert_allclose(bv["sk"], skb, rtol=1e-11)
    se = st.se()
    np.testing.assert_allclose(se["var"], D.var(axis=1).std(axis=0, ddof=1) / np.sqrt(B), rtol=1e-10)
    np.testing.assert_allclose(se["spatial_var"], D.var(axis=2).mean(axis=1).std(ddof=1) / np.sqrt(B), rtol=1e-10)
    # the whole-run statistics still use every sample
    np.testing.assert_allclose(st.spatial()[2], (X - ref).var(axis=1).mean(), atol=1e-14)


def test_batch_means_error_is_the_spread_of_independent_runs():
    """The batch-means SE estimates the standard deviation of a run's time
    average: over 40 independent realisations of the same periodic FE run
    (correlated samples: the slowest mode decays over ~33 steps, samples every
    25), the spread of their spatial-variance estimates agrees with the mean
    reported SE (a mis-scaled SE, e.g. without the 1/sqrt(B), is off by 4.5x),
    and fewer than two complete batches give NaN."""
    N, r = 16, 0.2
    est, ses = [], []
    for q in range(40):
        # no initial perturbation: the conserved mean, and with it the
        # stationary variance eps m^2 gamma / (1 - eps beta), is the same in
        # every realisation, so their spread is the sampling error alone
        d = oracle.Desc(dim=1, n=(N, 1, 1), r=r, sigma=oracle.sigma_of(r, 1e-2), u0=1.0, realisation=q, seed=21)
        u = oracle.init(d)
        oracle.advance(d, u, 0, 500)
        st = oracle.Stats(d, burn_in=500, every=25, per_cell=False, batch=30, max_batches=20)
        oracle.advance(d, u, 500, 500 + 25 * 600, st)
        assert st.n_batches == 20
        est.append(st.spatial()[2])
        ses.append(st.se()["spatial_var"])
    spread = np.std(est, ddof=1)
    ratio = spread / np.mean(ses)
    assert 0.7 < ratio < 1.4, ratio
    d = oracle.Desc(dim=1, n=(N, 1, 1), r=r, sigma=0.1, u0=1.0)
    st = oracle.Stats(d, burn_in=0, every=1, batch=10)
    oracle.advance(d, oracle.init(d), 0, 15, st)
    assert st.n_batches == 1 and np.all(np.isnan(st.se()["var"]))
