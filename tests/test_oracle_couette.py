"""Thermal Couette flow of Sec. VI.A on the oracle (CPU only).

Walls normal to y, the top one moving at u0 along x, both at T = 1; the
paper's own wall condition (a KBC/NEEP hybrid) is not specified, so the
walls reflect diffusely (what reaches a wall in a step leaves it at the
wall's velocity and temperature, with the density that returns the same
mass).  Such a wall slips by about one mean free path, so the closed forms
are checked on the slip-corrected gap:

* mass is conserved exactly;
* the steady profile is linear and symmetric, with slip u_s at each wall;
* the impulsive start follows the Stokes series (Eq. CouetteVelocity) with
  the lattice viscosity on the effective gap L + 2 l_s;
* viscous heating: the steady temperature is a parabola with
  T'' = -2 Pr (du/dy)^2 / (D + N_f + 2), the dimensionless form of
  Eq. Couette (C_p = (D + N_f + 2)/2), which pins Pr and N_f.
"""
import numpy as np
import pytest

import oracle

R, L = 3, 64                     # ghost rows per wall, gas rows


def couette(u0, steps, tau=1.0, Pr=0.71, Nf=3, nx=4, threads=4):
    prev = oracle.set_threads(0)
    oracle.set_threads(threads)
    try:
        ny = L + 2 * R
        sim = oracle.Sim(2, 37, Nf, Pr, tau, (nx, ny))
        sim.init(np.ones((ny, nx)), np.zeros((2, ny, nx)), np.ones((ny, nx)))
        sim.set_walls((0.0, 0.0, 1.0), (u0, 0.0, 1.0))
        t0 = sim.totals()
        out = []
        for s in steps:
            sim.step(s - sim.steps)
            m = sim.moments()
            out.append((m["u"][0].mean(1)[R:ny - R], m["T"].mean(1)[R:ny - R], sim.totals()))
        return t0, out
    finally:
        oracle.set_threads(prev)


def nu_lattice(tau):
    r = oracle.Lattice(2, 37).r
    return (tau - 0.5) / r ** 2            # cells^2 per step at T = 1


def stokes_series(y, nu, t, gap):
    n = np.arange(1, 400)[:, None]
    return y + 2 / np.pi * np.sum((-1.0) ** n / n * np.exp(-(n * np.pi) ** 2 * nu * t / gap ** 2)
                                  * np.sin(n * np.pi * y), axis=0)


def test_couette_mass_slip_and_stokes_transient():
    u0, tau = 0.1, 1.0
    t0, out = couette(u0, [500, 2000, 40000], tau=tau)
    for _, _, tot in out:
        assert abs(tot[0] - t0[0]) / t0[0] < 1e-11                    # walls return what they receive (FP64 rounding over 4e4 steps)
    rows = np.arange(L) + 0.5                                          # gas cell centres; walls at 0 and L
    u_inf = out[-1][0] / u0
    b, a = np.polyfit(rows, u_inf, 1)
    assert np.max(np.abs(u_inf - (a + b * rows))) < 2e-4               # linear
    slip_bottom, slip_top = a, 1 - (a + b * L)
    assert abs(slip_bottom - slip_top) < 1e-4                          # symmetric
    ls = a / b                                                         # slip length in cells
    mfp = nu_lattice(tau) * oracle.Lattice(2, 37).r                    # nu / c with c = 1/r cells per step
    assert 0.8 < ls / mfp < 2.0, (ls, mfp)
    gap = L + 2 * ls
    y = (rows + ls) / gap
    for (u, _, _), t in zip(out[:2], (500, 2000)):
        err = np.max(np.abs(u / u0 - stokes_series(y, nu_lattice(tau), t, gap)))
        assert err < 4e-3, (t, err)


def test_couette_viscous_heating_sets_prandtl_and_cp():
    for Pr, Nf in ((0.71, 3), (2.0, 1)):
        u0, tau = 0.3, 1.0
        _, out = couette(u0, [60000], tau=tau, Pr=Pr, Nf=Nf)
        u, T, _ = out[-1]
        rows = np.arange(L) + 0.5
        du = np.polyfit(rows, u, 1)[0]
        c2 = np.polyfit(rows, T - 1, 2)[0]
        want = -Pr * du ** 2 / (2 + Nf + 2)
        assert abs(c2 / want - 1) < 0.03, (Pr, Nf, c2, want)


def test_conduction_between_walls_at_different_temperatures():
    """Walls at rest at T = 1 and 1.02: the steady gas temperature is linear
    between them (a temperature jump of similar size at each wall, as the
    velocity slip), the gas at rest, and T_tr = T_int: the internal energy
    population takes the wall temperature too."""
    prev = oracle.set_threads(0)
    oracle.set_threads(4)
    try:
        nx, ny, Tt = 4, L + 2 * R, 1.02
        sim = oracle.Sim(2, 37, 3, 0.71, 1.0, (nx, ny))
        sim.init(np.ones((ny, nx)), np.zeros((2, ny, nx)), np.ones((ny, nx)))
        sim.set_walls((0.0, 0.0, 1.0), (0.0, 0.0, Tt))
        sim.step(60000)
        m = sim.moments(with_P=True)
    finally:
        oracle.set_threads(prev)
    rows = np.arange(L) + 0.5
    T = m["T"].mean(1)[R:ny - R]
    b, a = np.polyfit(rows, T, 1)
    assert np.max(np.abs(T - (a + b * rows))) < 3e-6 * L                 # linear (rho T = p uniform)
    jb, jt = a - 1.0, Tt - (a + b * L)
    assert jb > 0 and jt > 0 and abs(jb / jt - 1) < 0.05                 # symmetric jumps
    assert 0.9 < b * L / (Tt - 1) < 1.0                                  # most of the drop inside the gas
    # at rest beyond the walls' kinetic layer: the cells next to a wall hold
    # wall-emitted particles in transit (1e-5 at the first row, alternating
    # in sign and decaying by about 2 per row)
    assert np.max(np.abs(m["u"][:, 6 * R:ny - 6 * R])) < 1e-8   # decays over about 10 rows
    assert np.max(np.abs(m["u"])) < 1e-3 * (Tt - 1)
    p = m["rho"].mean(1)[R:ny - R] * T
    assert np.max(np.abs(p / p.mean() - 1)) < 1e-4                       # uniform pressure
