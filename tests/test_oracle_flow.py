"""Simulation-level pins of the FP64 oracle (CPU only): closed-form decay of
the shear and entropy modes (linearised Navier-Stokes with the transport
coefficients the scheme is built to give: kinematic viscosity
nu = (T/r^2)(tau - 1/2) in grid units and thermal diffusivity nu/Pr),
second-order convergence of those rates, exact conservation, and the
symmetries of the periodic lattice."""
import numpy as np
import pytest

import oracle
import workloads

KAPPA = 0.2


def decay_rates(n, steps, every, Pr=0.71, tau=0.8, Nf=3):
    D = 2
    sim = oracle.Sim(D, 37, Nf, Pr, tau, (n, n), kappa=KAPPA)
    rho, u, T = workloads.decay_2d(n)
    sim.init(rho, u, T)
    gamma = (Nf + D + 2) / (Nf + D)
    yy, xx = np.mgrid[0:n, 0:n]
    s_y = np.sin(2 * np.pi * yy / n)
    c_x = np.cos(2 * np.pi * xx / n)
    ts, As, AT = [], [], []
    for t in range(0, steps + 1, every):
        if t:
            sim.step(every)
        m = sim.moments()
        p = m["rho"] * m["T"]
        E = (m["T"] - 1) - (gamma - 1) / gamma * (p - 1)      # entropy mode, acoustic part removed
        ts.append(t)
        As.append(2 * np.mean(m["u"][0] * s_y))
        AT.append(2 * np.mean(E * c_x))
    ts = np.array(ts, float)
    sel = ts >= steps * 0.2
    lam_s = -np.polyfit(ts[sel], np.log(np.array(As)[sel]), 1)[0]
    lam_T = -np.polyfit(ts[sel], np.log(np.array(AT)[sel]), 1)[0]
    r = oracle.Lattice(2, 37).r
    k2 = (2 * np.pi / n) ** 2
    nu = (tau - 0.5) / r ** 2
    return lam_s / (nu * k2) - 1, lam_T / (nu / Pr * k2) - 1, AT[0]


def test_decay_rates_match_closed_form_and_converge():
    """Plain-method case: 32^2, tau = 0.8, Pr = 0.71, N_f = 3, 500 steps.
    Both rates within 1% of the closed form; halving the wavenumber (64^2,
    2000 steps) cuts the error by a factor 3..5 (second order)."""
    es32, eT32, A0 = decay_rates(32, 500, 10)
    assert abs(es32) < 0.01 and abs(eT32) < 0.01, (es32, eT32)
    # the entropy mode starts at 1e-3/gamma for a non-isobaric temperature wave
    assert abs(A0 - 1e-3 / 1.4) < 2e-6
    es64, eT64, _ = decay_rates(64, 2000, 40)
    assert 3.0 < es32 / es64 < 5.0, (es32, es64)
    assert 3.0 < eT32 / eT64 < 5.0, (eT32, eT64)


@pytest.mark.parametrize("Pr", [0.5, 2.0])
def test_prandtl_number_sets_thermal_decay(Pr):
    es, eT, _ = decay_rates(32, 400, 10, Pr=Pr, tau=0.7)
    assert abs(es) < 0.015 and abs(eT) < 0.015, (Pr, es, eT)


def test_conservation_and_translation():
    n = (24, 20)
    rho, u, T = workloads.random_state(n, seed=5)
    a = oracle.Sim(2, 37, 3, 0.71, 0.6, n, kappa=KAPPA)
    a.init(rho, u, T)
    t0 = a.totals()
    a.step(20)
    t1 = a.totals()
    np.testing.assert_allclose(t1, t0, rtol=1e-13, atol=1e-12)
    # periodic translation by (5, 3): results translate exactly
    sh = lambda f: np.roll(np.roll(f, 3, axis=-2), 5, axis=-1)
    b = oracle.Sim(2, 37, 3, 0.71, 0.6, n, kappa=KAPPA)
    b.init(sh(rho), sh(u), sh(T))
    b.step(20)
    ma, mb = a.moments(), b.moments()
    for k in ("rho", "u", "T"):
        assert np.array_equal(sh(ma[k]), mb[k])


def test_reflection_and_transpose_symmetry():
    n = 24
    rho, u, T = workloads.random_state((n, n), seed=6)
    a = oracle.Sim(2, 37, 1, 1.3, 0.7, (n, n), kappa=KAPPA)
    a.init(rho, u, T)
    a.step(15)
    ma = a.moments()
    # x -> -x: mirror fields, flip u_x
    mir = lambda f: np.roll(f[..., ::-1], 1, axis=-1)
    b = oracle.Sim(2, 37, 1, 1.3, 0.7, (n, n), kappa=KAPPA)
    b.init(mir(rho), np.stack([-mir(u[0]), mir(u[1])]), mir(T))
    b.step(15)
    mb = b.moments()
    np.testing.assert_allclose(mb["rho"], mir(ma["rho"]), rtol=1e-13)
    np.testing.assert_allclose(mb["T"], mir(ma["T"]), rtol=1e-13)
    np.testing.assert_allclose(mb["u"][0], -mir(ma["u"][0]), atol=1e-14)
    np.testing.assert_allclose(mb["u"][1], mir(ma["u"][1]), atol=1e-14)
    # x <-> y: transpose fields and swap velocity components
    c = oracle.Sim(2, 37, 1, 1.3, 0.7, (n, n), kappa=KAPPA)
    c.init(rho.T.copy(), np.stack([u[1].T, u[0].T]).copy(), T.T.copy())
    c.step(15)
    mc = c.moments()
    np.testing.assert_allclose(mc["rho"], ma["rho"].T, rtol=1e-13)
    np.testing.assert_allclose(mc["u"][0], ma["u"][1].T, atol=1e-14)


@pytest.mark.parametrize("D,Q,Nf", [(2, 37, 3), (3, 39, 2), (2, 37, 0)])
def test_uniform_state_is_fixed_point(D, Q, Nf):
    dims = (6,) * D
    shape = dims
    sim = oracle.Sim(D, Q, Nf, 0.71, 0.7, dims, kappa=KAPPA)
    sim.init(np.full(shape, 1.3), np.zeros((D,) + shape), np.full(shape, 0.9))
    f0, g0 = sim.get_pops()
    sim.step(7)
    f1, g1 = sim.get_pops()
    np.testing.assert_allclose(f1, f0, rtol=1e-13)
    if Nf:
        np.testing.assert_allclose(g1, g0, rtol=1e-13)


def _tgv_rate_error(n, tau=0.7):
    """Relative error of the kinetic-energy decay rate of a D3Q39 Taylor-Green
    vortex against 6 nu k0^2 (k0 = 2 pi/n), measured over the second half of
    a run lasting one decay time scale, after the initial layer."""
    steps = int(round(40 * (n / 24) ** 2))
    sim = oracle.Sim(3, 39, 2, 0.71, tau, (n, n, n), kappa=KAPPA)
    rho, u, T = workloads.taylor_green_3d(n, u0=0.01, amp_T=0.0)
    sim.init(rho, u, T)
    t0 = sim.totals()

    def ke():
        m = sim.moments()
        return 0.5 * float(np.sum(m["rho"] * (m["u"] ** 2).sum(0)))

    sim.step(steps // 2)
    k1 = ke()
    sim.step(steps - steps // 2)
    k2 = ke()
    # totals are plain sums over ~1e6 values: their own rounding is ~1e-12
    np.testing.assert_allclose(sim.totals(), t0, rtol=1e-11, atol=1e-11)
    r = oracle.Lattice(3, 39).r
    nu = (tau - 0.5) / r ** 2
    rate = -np.log(k2 / k1) / (steps - steps // 2)
    return rate / (6 * nu * (2 * np.pi / n) ** 2) - 1


def test_taylor_green_3d_kinetic_energy_decay():
    """D3Q39 Taylor-Green vortex at low Mach number (no temperature wave,
    whose sound would dominate once the vortex has decayed): the decay rate
    of the kinetic energy is 6 nu k0^2 to within 4% at 24^3, and the error
    falls as k0^2 (24^3 -> 32^3), with totals conserved."""
    e24 = _tgv_rate_error(24)
    e32 = _tgv_rate_error(32)
    assert abs(e24) < 0.04 and abs(e32) < 0.025, (e24, e32)
    assert 1.4 < e24 / e32 < 2.3, (e24, e32)
