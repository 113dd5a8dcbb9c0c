"""Acoustic pin of the oracle (CPU only): a small pressure wave travels at
the adiabatic sound speed sqrt(gamma T) (thermal units; sqrt(gamma T)/r
cells per step), with gamma = (N_f + D + 2)/(N_f + D) (Eq. Gamma).  This is
what N_f controls; the shear and entropy decays do not see it.  The
frequency error falls as k^2."""
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
