"""Acoustic pins of the oracle (CPU only).

* A small pressure wave travels at the adiabatic sound speed sqrt(gamma T)
  (thermal units; sqrt(gamma T)/r cells per step), with
  gamma = (N_f + D + 2)/(N_f + D) (Eq. Gamma).  This is what N_f controls; the
  shear and entropy decays do not see it.  The frequency error falls as k^2.
* Its amplitude decays at Gamma = (k^2/2)[2(1 - 1/D) nu + zeta/rho +
  (gamma - 1) chi], the linearised Navier-Stokes attenuation with the lattice
  transport coefficients (grid units, c^2 = T/r^2): shear viscosity
  nu = c^2 (1/omega_s - 1/2), thermal diffusivity chi = c^2 (1/omega - 1/2),
  and the bulk viscosity of the exchange between translational and internal
  energy.  That exchange relaxes T_tr - T_int at kappa omega per step (the
  trace of Lambda pulls T_tr toward T_eq with weight kappa, Sec. II, and
  T_rel pulls T_int the same way), so zeta/rho = c^2 2 N_f/(D (D + N_f))
  (1/(kappa omega) - 1/2).  The paper states the second viscosity of the
  continuous model only for its literal rates (Sec. II); this is the same
  Chapman-Enskog argument for the rates the library uses.  This pins kappa.
"""
import numpy as np
import pytest

import oracle


def sound_speed_error(Nf, n, periods=4, tau=0.8, Pr=0.71):
    D, ny = 2, 4
    gamma = (Nf + D + 2) / (Nf + D)
    r = oracle.Lattice(2, 37).r
    cs = np.sqrt(gamma) / r
    steps = int(periods * n / cs)
    sim = oracle.Sim(2, 37, Nf, Pr, tau, (n, ny))
    x = np.tile(np.arange(n, dtype=float), (ny, 1))
    sim.init(1 + 1e-4 * np.cos(2 * np.pi * x / n), np.zeros((2, ny, n)), np.ones((ny, n)))
    c = np.cos(2 * np.pi * x / n)
    amp = []
    for _ in range(steps + 1):
        m = sim.moments()
        amp.append(2 * np.mean((m["rho"] * m["T"] - 1) * c))   # pressure: the entropy mode carries none
        sim.step(1)
    a = np.array(amp)
    zc = [i + a[i] / (a[i] - a[i + 1]) for i in range(len(a) - 1) if a[i] * a[i + 1] < 0]
    period = 2 * np.mean(np.diff(zc))
    return (n / period) / cs - 1


@pytest.mark.parametrize("Nf", [0, 1, 3])
def test_sound_speed_sets_gamma(Nf):
    e = sound_speed_error(Nf, 128)
    assert abs(e) < 0.012, (Nf, e)


def test_sound_speed_converges_second_order():
    e64, e128 = sound_speed_error(3, 64), sound_speed_error(3, 128)
    assert 3.0 < e64 / e128 < 5.0, (e64, e128)


def fit_attenuation(samples, k, cs, skip=20):
    """Damped-cosine fit A exp(-G t) cos(w t + p) of a pressure-mode history."""
    from scipy.optimize import curve_fit
    a = np.asarray(samples)
    t = np.arange(len(a))
    sel = t > skip
    f = lambda t, A, G, w, p: A * np.exp(-G * t) * np.cos(w * t + p)
    popt, _ = curve_fit(f, t[sel], a[sel], p0=[a[sel][0], 1e-3, cs * k, 0.0], maxfev=20000)
    return popt[1], popt[2]


def predicted_attenuation(Nf, kappa, tau, Pr, n, D=2):
    r = oracle.Lattice(2, 37).r
    gamma = (Nf + D + 2) / (Nf + D)
    k = 2 * np.pi / n
    om_s, om = 1 / tau, 1 / (0.5 + (tau - 0.5) / Pr)
    c2 = 1 / r ** 2
    nu, chi = c2 * (1 / om_s - 0.5), c2 * (1 / om - 0.5)
    zeta = c2 * 2 * Nf / (D * (D + Nf)) * (1 / (kappa * om) - 0.5) if Nf > 0 else 0.0
    return 0.5 * k ** 2 * (2 * (1 - 1 / D) * nu + zeta + (gamma - 1) * chi)


@pytest.mark.parametrize("Nf,kappa,Pr", [(0, 0.2, 1.0), (1, 0.25, 1.0), (3, 0.25, 1.0), (3, 0.5, 1.0),
                                         (3, 0.9, 1.0), (3, 0.2, 0.71), (3, 0.5, 2.0)])
def test_sound_attenuation_sets_bulk_viscosity(Nf, kappa, Pr):
    n, ny, tau, D = 256, 4, 0.8, 2
    r = oracle.Lattice(2, 37).r
    cs = np.sqrt((Nf + D + 2) / (Nf + D)) / r
    sim = oracle.Sim(2, 37, Nf, Pr, tau, (n, ny), kappa=kappa)
    x = np.tile(np.arange(n, dtype=float), (ny, 1))
    sim.init(1 + 1e-4 * np.cos(2 * np.pi * x / n), np.zeros((2, ny, n)), np.ones((ny, n)))
    c = np.cos(2 * np.pi * x / n)
    amp = []
    for _ in range(int(6 * n / cs) + 1):
        m = sim.moments()
        amp.append(2 * np.mean((m["rho"] * m["T"] - 1) * c))
        sim.step(1)
    G, w = fit_attenuation(amp, 2 * np.pi / n, cs)
    Gp = predicted_attenuation(Nf, kappa, tau, Pr, n)
    assert abs(G / Gp - 1) < 0.015, (Nf, kappa, Pr, G, Gp)
    assert abs(w / (cs * 2 * np.pi / n) - 1) < 0.003
