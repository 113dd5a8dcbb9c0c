"""Pins of the oracle's collision and parameter mapping (CPU only).

The collision is checked through what the scheme must do to moments, not by
retyping it: exact conservation of mass, momentum and energy; relaxation of
the deviatoric stress at the stress rate; of the heat flux at the heat-flux
rate; and of the translational/internal temperature split toward T_eq with
weight kappa (the T_rel target of Eq. ReductionH)."""
import numpy as np
import pytest

import oracle

KAPPA = 0.2


def random_nonequilibrium(L, Nf, n, rng, amp=0.05):
    """Equilibrium populations of random (rho, u, T) with random
    perturbations proportional to the weights."""
    D, Q = L.D, L.Q
    f = np.zeros((n, Q))
    g = np.zeros((n, Q)) if Nf > 0 else None
    for k in range(n):
        rho = rng.uniform(0.9, 1.1)
        u = rng.uniform(-0.1, 0.1, D)
        T = rng.uniform(0.95, 1.05)
        G = oracle.equilibrium(D, Q, rho, u, (T - 1) * np.eye(D))
        f[k] = G + L.w * amp * rng.standard_normal(Q)
        if Nf > 0:
            g[k] = 0.5 * Nf * rng.uniform(0.95, 1.05) * G + L.w * amp * rng.standard_normal(Q)
    return f, g


def cell_stats(L, Nf, f, g):
    """Moments of one cell computed here, independently of the oracle."""
    xi = L.xi
    rho = f.sum()
    u = (xi * f[:, None]).sum(0) / rho
    c = xi - u
    sig = (c[:, :, None] * c[:, None, :] * f[:, None, None]).sum(0) / rho
    Ttr = np.trace(sig) / L.D
    q = 0.5 * ((c ** 2).sum(1)[:, None] * c * f[:, None]).sum(0)
    en = 0.5 * ((xi ** 2).sum(1) * f).sum()
    Tint = None
    if Nf > 0:
        q = q + (c * g[:, None]).sum(0)
        en += g.sum()
        Tint = 2 * g.sum() / (Nf * rho)
    return dict(rho=rho, j=rho * u, u=u, sig=sig, Ttr=Ttr, q=q, en=en, Tint=Tint)


CASES = [(2, 37, 3, 0.71, 0.6), (2, 37, 0, 2.0, 0.9), (2, 37, 1, 0.5, 1.2), (3, 39, 2, 0.71, 0.7),
         (2, 33, 3, 0.71, 2 / 3)]


@pytest.mark.parametrize("D,Q,Nf,Pr,tau", CASES)
def test_collision_conserves_and_relaxes(D, Q, Nf, Pr, tau):
    L = oracle.Lattice(D, Q)
    rng = np.random.default_rng(D * 1000 + Q * 10 + Nf)
    f, g = random_nonequilibrium(L, Nf, 4, rng)
    fo, go = oracle.collide_cells(D, Q, Nf, Pr, tau, KAPPA, f, g)
    pm = oracle.param_map(D, Nf, Pr, tau, KAPPA)
    om, oms = pm["omega"], pm["omega_s"]
    for k in range(f.shape[0]):
        a = cell_stats(L, Nf, f[k], g[k] if Nf else None)
        b = cell_stats(L, Nf, fo[k], go[k] if Nf else None)
        # conservation (Section V moments)
        assert abs(b["rho"] - a["rho"]) < 1e-14
        np.testing.assert_allclose(b["j"], a["j"], atol=1e-15)
        assert abs(b["en"] - a["en"]) < 2e-14
        # deviatoric stress relaxes at the stress rate
        dev = lambda s: s - np.trace(s) / D * np.eye(D)
        np.testing.assert_allclose(dev(b["sig"]) * b["rho"], (1 - oms) * dev(a["sig"]) * a["rho"], atol=1e-13)
        # heat flux relaxes at the heat-flux rate (the Gaussian carries none)
        np.testing.assert_allclose(b["q"], (1 - om) * a["q"], atol=1e-13)
        # temperature exchange toward T_eq with weight kappa
        Teq = (D * a["Ttr"] + Nf * (a["Tint"] if Nf else a["Ttr"])) / (D + Nf)
        assert abs(b["Ttr"] - (a["Ttr"] - om * KAPPA * (a["Ttr"] - Teq))) < 1e-13
        if Nf > 0:
            assert abs(b["Tint"] - (a["Tint"] - om * KAPPA * (a["Tint"] - Teq))) < 1e-13


@pytest.mark.parametrize("D,Q,Nf", [(2, 37, 3), (3, 39, 2)])
def test_equilibrium_is_fixed_point_of_collision(D, Q, Nf):
    L = oracle.Lattice(D, Q)
    rho, u, T = 1.2, np.full(D, 0.05), 1.1
    G = oracle.equilibrium(D, Q, rho, u, (T - 1) * np.eye(D))
    fo, go = oracle.collide_cells(D, Q, Nf, 0.71, 0.8, KAPPA, G[None], (0.5 * Nf * T * G)[None])
    np.testing.assert_allclose(fo[0], G, rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(go[0], 0.5 * Nf * T * G, rtol=1e-13, atol=1e-16)


def test_reading_b_gives_exact_lattice_prandtl_number():
    """Reading B: stress rate 1/tau, heat-flux rate omega with
    (1/omega_s - 1/2) / (1/omega - 1/2) = Pr for every tau > 1/2."""
    for Pr in (0.5, 0.71, 1.0, 2.0):
        for tau in (0.55, 0.6, 0.8, 1.2, 5.0):
            p = oracle.param_map(2, 3, Pr, tau, KAPPA)
            assert abs(p["omega_s"] - 1 / tau) < 1e-15
            assert abs((1 / p["omega_s"] - 0.5) / (1 / p["omega"] - 0.5) - Pr) < 1e-12
            # the ES parameter reproduces the stress rate: omega_s = omega (1 - (1 - kappa) nu)
            assert abs(p["omega"] * (1 - (1 - KAPPA) * p["nu"]) - p["omega_s"]) < 1e-14
            assert 0 < p["omega"] < 2


def test_reading_b_tends_to_paper_relations_for_large_tau():
    """For tau -> infinity reading B's rate is Pr/tau (Eq. DiscreteReductionG)
    and nu satisfies Pr = 1/(1 - nu + kappa nu) (Eq. Pr)."""
    for Pr in (0.5, 0.71, 2.0):
        tau = 1e7
        p = oracle.param_map(2, 3, Pr, tau, KAPPA)
        assert abs(p["omega"] * tau / Pr - 1) < 1e-6
        assert abs(1 / (1 - p["nu"] + KAPPA * p["nu"]) - Pr) < 1e-6
        pa = oracle.param_map(2, 3, Pr, tau, KAPPA, reading="A")
        assert abs(pa["omega"] - Pr / tau) < 1e-20
        assert abs(1 / (1 - pa["nu"] + KAPPA * pa["nu"]) - Pr) < 1e-12


def test_bgk_limit_at_unit_prandtl_number():
    p = oracle.param_map(2, 3, 1.0, 0.8, KAPPA)
    assert abs(p["nu"]) < 1e-15 and abs(p["omega"] - 1 / 0.8) < 1e-15


def test_specific_heat_ratio():
    """gamma = (N_f + D + 2)/(N_f + D) (Eq. Gamma)."""
    assert abs(oracle.param_map(2, 3, 0.71, 0.8)["gamma"] - 1.4) < 1e-15
    assert abs(oracle.param_map(3, 2, 0.71, 0.8)["gamma"] - 1.4) < 1e-15
    assert abs(oracle.param_map(2, 0, 0.71, 0.8)["gamma"] - 2.0) < 1e-15
    assert abs(oracle.param_map(2, 1, 0.71, 0.8)["gamma"] - 5 / 3) < 1e-15


def test_couette_example_parameters_need_negative_nu():
    """Section VI.A quotes Pr = 0.71 for kappa = 0.2 and nu = 0.5; Eq. Pr
    gives 0.714 only for nu = -0.5 (the printed sign is read as a typo)."""
    pr = lambda nu, k: 1 / (1 - nu + k * nu)
    assert abs(pr(-0.5, 0.2) - 0.714) < 1e-3
    assert abs(pr(0.5, 0.2) - 1.667) < 1e-3


@pytest.mark.parametrize("bad", [dict(tau=0.5), dict(Pr=0.0), dict(Nf=-1), dict(kappa=1.0)])
def test_invalid_parameters_rejected(bad):
    args = dict(D=2, Nf=3, Pr=0.71, tau=0.8, kappa=KAPPA)
    args.update(bad)
    with pytest.raises(ValueError):
        oracle.param_map(**args)
