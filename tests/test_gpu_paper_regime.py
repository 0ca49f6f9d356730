"""The paper's worked example on the GPU: the iron rod of Sec. 3 (N = 32
cells, predictor-corrector at the program's a = 1/10, Dirichlet walls), with
the printed constants of tests/golden/iron_rod.json converted as in
tests/test_paper_regime.py.

  * Equilibrium at 300 K for the paper's 2e6 steps (FP64 state) and the
    100 K / 500 K gradient for its 8e6 steps (FP32 state, FP64 statistics),
    sampled every 10 steps after 10% relaxation, as the supplementary program
    does: mean, variance, covariance, S_k and their batch-means error bars
    against the oracle on the same noise.
  * The same runs against the scheme's own exact statistics: the linear
    profile is the exact mean; the equilibrium variance is the discrete
    Lyapunov value (within 1% of the paper's k_B T^2 / (rho c_V dV) of eq.
    varcorrT_EQ at this time step).
  * A 512-realisation ensemble of the gradient run with the deterministic
    face temperature in the noise (the scheme is then linear): its covariance
    equals the discrete Lyapunov solution element by element, which resolves
    the long-range correlation of eq. TcorrNEQ (1.4% of the diagonal at the
    centre) in the column x_j = L/4 the paper plots.
"""
import numpy as np
import pytest

import oracle
import theory
from helpers import gpu_instance, max_rel, oracle_desc
from paper_2406_12157_amd import workloads as W
from test_paper_regime import GOLD, regime

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def she():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2406_12157_amd import she as mod
    mod.load()
    return mod


def iron(tl, tr, noise=0, realisation=0):
    N, r, eps, _ = regime()
    tm = 0.5 * (tl + tr)
    return W.instance((N,), bc=W.DIRICHLET, scheme=W.HEUN, noise=noise, r=r, eps=eps, u0=tm, u_left=tl,
                      u_right=tr, init_sd=np.sqrt(eps) * tm, seed=2024, realisation=realisation)


@pytest.mark.parametrize("case", ["equilibrium", "gradient"])
def test_iron_rod_against_the_oracle_and_the_scheme(she, case):
    N, r, eps, _ = regime()
    if case == "equilibrium":
        tl = tr = GOLD["T_eq"]
        steps, prec, tol, se_tol = GOLD["steps_equilibrium"], 1, 1e-9, 1e-9
    else:
        tl, tr = GOLD["T_left_gradient"], GOLD["T_right_gradient"]
        # FP32 state over 8e6 steps: the trajectories differ by rounding, a
        # few 1e-5 of the fluctuation; the error bars, a spread of batch
        # values, take that relative to the spread (1e-2)
        steps, prec, tol, se_tol = GOLD["steps_gradient"], 0, 1e-3, 1e-2
    every, burn = 10, steps // 10
    L = (steps - burn) // every // 20           # 20 batches
    inst = iron(tl, tr)
    h = she.Handle([gpu_instance(she, inst)], precision=prec, burn_in=burn, sample_every=every,
                   stats=she.STAT_MOMENTS | she.STAT_CORR, batch_samples=L)
    u = h.read_field(0)
    h.run(steps)
    g = h.stats(0, corr=True, sk=True, se=True)
    h.close()
    d = oracle_desc(inst, prec)
    st = oracle.Stats(d, burn_in=burn, every=every, corr=True, batch=L)
    oracle.advance(d, u, 0, steps, st)
    assert g["n_samples"] == st.n_samples == (steps - burn) // every
    assert g["n_batches"] == st.n_batches == 20
    se = st.se()
    cov = st.cov()
    assert max_rel(g["mean"], st.mean()) < tol
    assert max_rel(g["var"], st.var()) < tol
    assert np.max(np.abs(g["corr"] - cov)) < tol * np.max(np.diag(cov))
    for key in ("mean", "var"):
        assert max_rel(g[key + "_se"], se[key]) < se_tol, key
    assert abs(g["spatial_var"] / st.spatial()[2] - 1) < tol
    # the scheme's exact statistics: mean = the linear profile (exact fixed
    # point), covariance = the discrete Lyapunov solution for the face
    # amplitude of that profile (instantaneous amplitudes add O(eps) = 0.2%)
    ref = oracle.reference(d)
    assert np.all(np.abs(g["mean"] - ref) <= 4.5 * g["mean_se"] + 1e-9 * np.abs(ref))
    G, B = theory.dirichlet_operators(N, r, oracle.sigma_of(r, eps), tl, tr, "pc")
    C = theory.discrete_lyapunov(G, B)
    rel = g["var"] / np.diag(C) - 1.0
    assert np.all(np.abs(rel) <= 5e-3 + 4.5 * g["var_se"] / np.diag(C)), rel
    if case == "equilibrium":
        paper = eps * tl * tl                   # eq. varcorrT_EQ: k_B T^2 / (rho c_V dV) = 140.3 K^2
        assert abs(np.mean(np.diag(C)) / paper - 1) < 0.01
        assert abs(np.mean(g["var"]) / paper - 1) < 0.01 + 4.5 * np.sqrt(np.mean(g["var_se"] ** 2) / N) / paper


def test_iron_rod_gradient_ensemble_resolves_the_long_range_correlation(she):
    N, r, eps, _ = regime()
    tl, tr = GOLD["T_left_gradient"], GOLD["T_right_gradient"]
    Q, steps, every = 512, 2000000, 10
    insts = [iron(tl, tr, noise=1, realisation=q) for q in range(Q)]
    h = she.Handle([gpu_instance(she, i) for i in insts], precision=0, burn_in=steps // 10, sample_every=every,
                   stats=she.STAT_MOMENTS | she.STAT_CORR)
    h.run(steps)
    ref = oracle.reference(oracle_desc(insts[0], 0))
    # second moments about the exact mean (the linear profile), per realisation
    mom = []
    for q in range(Q):
        g = h.stats(q, corr=True)
        dm = g["mean"] - ref
        mom.append(g["corr"] + np.outer(dm, dm))
    h.close()
    mom = np.array(mom)
    C_gpu = mom.mean(axis=0)
    se = mom.std(axis=0, ddof=1) / np.sqrt(Q)
    G, B = theory.dirichlet_operators(N, r, oracle.sigma_of(r, eps), tl, tr, "pc")
    C = theory.discrete_lyapunov(G, B)
    scale = np.max(np.diag(C))
    z = np.abs(C_gpu - C) / (se + 1e-3 * scale)
    assert np.max(z) < 4.5, np.max(z)
    # the paper's eq. TcorrNEQ in the plotted column, off the diagonal: the
    # long-range part is resolved (signal over error) and follows the theory
    tbar = tl + (tr - tl) * (np.arange(N) + 0.5) / N
    want = theory.garcia_neq_correlation(N, eps, tbar, tr - tl)
    j = N // 4
    off = np.abs(np.arange(N) - j) >= 2
    amp = np.max(np.abs(want[off, j]))
    assert amp / np.mean(np.diag(want)) > 0.005
    assert np.median(np.abs(C_gpu[off, j]) / se[off, j]) > 5
    assert np.max(np.abs(C_gpu[off, j] - want[off, j])) < 0.1 * amp + 4.5 * np.max(se[off, j])
