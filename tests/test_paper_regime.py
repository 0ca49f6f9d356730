"""The paper's own worked example (iron rod, Sec. 3), with its printed
constants from ``tests/golden/iron_rod.json``: the oracle run in that regime
reproduces the equilibrium variance k_B T^2/(rho c_V dV) of eq. varcorrT_EQ
(the PC scheme at the program's a = 1/10 is within 1% of it, Sec. 3 remark that
PC agrees better), and the nondimensional numbers follow from the constants.
"""
import json
import os

import numpy as np

import oracle
import theory

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "iron_rod.json")))


def regime():
    g = GOLD
    N = g["N"]
    dx = g["length"] / N
    dv = g["area"] * dx
    kappa = g["lambda"] / (g["rho"] * g["c_V"])
    dt = g["stability_factor_a"] * dx * dx / (2 * kappa)
    r = kappa * dt / dx ** 2
    eps = g["k_B"] / (g["rho"] * g["c_V"] * dv)
    return N, r, eps, dt


def test_nondimensional_numbers():
    N, r, eps, dt = regime()
    g = GOLD
    assert abs(r - g["stability_factor_a"] / 2) < 1e-15       # dt = a dx^2 / (2 kappa)
    atoms = g["rho"] * g["length"] * g["area"] / g["m_atom"]
    assert 0.3 * g["atoms_order_of_magnitude"] < atoms < 3 * g["atoms_order_of_magnitude"]
    assert atoms / N > 10                                      # O(10) molecules per cell or more
    var300 = eps * g["T_eq"] ** 2
    assert 100 < var300 < 200                                  # ~ (12 K)^2


def test_equilibrium_variance_paper_regime():
    N, r, eps, _ = regime()
    t0 = GOLD["T_eq"]
    d = oracle.Desc(dim=1, n=(N, 1, 1), bc=1, scheme=1, r=r, sigma=oracle.sigma_of(r, eps),
                    u_left=t0, u_right=t0, init_sd=np.sqrt(eps) * t0, seed=2024)
    u = oracle.init(d)
    oracle.advance(d, u, 0, 20000)
    vals = []
    for b in range(10):
        st = oracle.Stats(d, burn_in=0, every=10)
        oracle.advance(d, u, 20000 + b * 40000, 40000, st)
        vals.append(st.var().mean())
    v, se = np.mean(vals), np.std(vals, ddof=1) / np.sqrt(len(vals))
    paper = eps * t0 ** 2
    G, B = theory.dirichlet_operators(N, r, oracle.sigma_of(r, eps), t0, t0, "pc")
    exact = np.diag(theory.discrete_lyapunov(G, B)).mean()
    assert abs(exact / paper - 1) < 0.01
    assert abs(v - exact) < 4.5 * se, (v, exact, se)
