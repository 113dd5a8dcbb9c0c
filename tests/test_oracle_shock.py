"""Shock tube of Sec. VI.B on the oracle (CPU only).

The paper's case: D2Q33, 1000 x 16, (rho, T, u) = (4, 1, 0) | (1, 1, 0),
N_f = 3 (gamma = 1.4), tau = 2/3, 174 steps (t ~ 0.15 in units of the tube
length).  The paper's ends are open; in 174 steps no wave travels more than
~250 cells, so a periodic tube (whose wrap is a mirrored second interface)
has exactly the open-tube solution on cells 250..750.

The exact solution (oracle/riemann.py) is pinned first by the conditions
that define it, then the lattice solution is compared with it."""
import numpy as np
import pytest

import oracle
from oracle import riemann

G = 1.4
LEFT, RIGHT = (4.0, 0.0, 4.0), (1.0, 0.0, 1.0)     # (rho, u, p), p = rho T


def test_exact_solution_satisfies_jump_conditions():
    ps, us = riemann.star_state(LEFT, RIGHT, G)
    rl, _, pl = LEFT
    rr, _, pr = RIGHT
    assert ps < pl and ps > pr          # left rarefaction, right shock
    s = np.linspace(-2.0, 2.0, 4001)
    rho, u, p = riemann.sample(LEFT, RIGHT, G, s)
    # the rarefaction is isentropic and keeps the Riemann invariant u + 2c/(gamma-1)
    fan = (s > -np.sqrt(G * pl / rl)) & (u < us - 1e-9) & (u > 1e-9)
    assert fan.sum() > 50
    np.testing.assert_allclose(p[fan] / rho[fan] ** G, pl / rl ** G, rtol=1e-12)
    c = np.sqrt(G * p / rho)
    np.testing.assert_allclose(u[fan] + 2 * c[fan] / (G - 1), 2 * np.sqrt(G * pl / rl) / (G - 1), rtol=1e-12)
    # pressure and velocity continuous across the contact
    i = np.argmax(s > us)
    assert abs(p[i - 1] - p[i]) < 1e-12 and abs(u[i - 1] - u[i]) < 1e-12
    # Rankine-Hugoniot across the right shock, in the shock frame
    j = np.argmax((s > us) & (rho < rho[i] - 1e-9))
    S = 0.5 * (s[j - 1] + s[j])
    r2, u2, p2 = rho[j - 1], u[j - 1], p[j - 1]
    m1, m2 = rr * (0 - S), r2 * (u2 - S)
    assert abs(m1 - m2) / abs(m1) < 2e-3                               # mass (S located to the grid)
    rs = rr * (ps / pr + (G - 1) / (G + 1)) / ((G - 1) / (G + 1) * ps / pr + 1)
    Sx = (rs * us) / (rs - rr)                                          # exact shock speed from mass flux
    mom1 = rr * (0 - Sx) ** 2 + pr
    mom2 = rs * (us - Sx) ** 2 + ps
    e1 = (0 - Sx) ** 2 / 2 + G / (G - 1) * pr / rr
    e2 = (us - Sx) ** 2 / 2 + G / (G - 1) * ps / rs
    assert abs(mom1 - mom2) < 1e-10 * mom1 and abs(e1 - e2) < 1e-10 * e1


def shock_tube(threads=4):
    prev = oracle.set_threads(0)
    oracle.set_threads(threads)
    try:
        nx, ny, steps = 1000, 16, 174
        sim = oracle.Sim(2, 33, 3, 0.71, 2 / 3, (nx, ny))
        x = np.tile(np.arange(nx, dtype=float), (ny, 1))
        sim.init(np.where(x < 500, 4.0, 1.0), np.zeros((2, ny, nx)), np.ones((ny, nx)))
        sim.step(steps)
        return sim.moments(), steps
    finally:
        oracle.set_threads(prev)


def test_d2q33_shock_tube_matches_exact_solution():
    m, steps = shock_tube()
    r = oracle.Lattice(2, 33).r
    assert abs(steps / (1000 * r) - 0.15) < 0.001            # the paper's time conversion
    xs = np.arange(1000, dtype=float)
    s = (xs - 499.5) * r / steps          # cells per step -> thermal-unit speed of each cell centre
    re, ue, pe = riemann.sample(LEFT, RIGHT, G, s)
    rho, u = m["rho"].mean(0), m["u"][0].mean(0)
    p = (m["rho"] * m["T"]).mean(0)
    assert np.max(np.abs(m["rho"] - rho)) < 1e-12            # one-dimensional
    sel = (xs > 250) & (xs < 750)
    e_rho = np.abs(rho - re)[sel].sum() / re[sel].sum()
    e_u = np.abs(u - ue)[sel].sum() / np.abs(ue[sel]).sum()
    print(f"shock tube L1: rho {e_rho:.3e} u {e_u:.3e}")
    assert e_rho < 0.03 and e_u < 0.04
    ps, us = riemann.star_state(LEFT, RIGHT, G)
    plateau = (s > us + 0.1) & (s < 1.45)                     # between contact and shock
    assert np.max(np.abs(p[plateau] / ps - 1)) < 0.015
    # shock position: where rho crosses halfway between the post-shock and right states
    rs = re[plateau].mean()
    k = np.argmax((xs > 650) & (rho < 0.5 * (rs + 1.0)))
    Sx = (rs * us) / (rs - 1.0)
    assert abs(xs[k] - (499.5 + Sx * steps / r)) < 3.0


def open_tube(steps_list, threads=4, open_x=True):
    """The shock tube with the paper's open ends: 1000 gas columns between
    zero-gradient ends (4 ghost columns each for D2Q33), one row."""
    prev = oracle.set_threads(0)
    oracle.set_threads(threads)
    try:
        RX, L = 4, 1000
        nx = L + 2 * RX
        sim = oracle.Sim(2, 33, 3, 0.71, 2 / 3, (nx, 1))
        x = np.arange(nx, dtype=float)[None, :] - RX
        sim.init(np.where(x < 500, 4.0, 1.0), np.zeros((2, 1, nx)), np.ones((1, nx)))
        if open_x:
            sim.set_open_x(True)
        out = []
        for s in steps_list:
            sim.step(s - sim.steps)
            m = sim.moments()
            out.append((s, m["rho"][0, RX:nx - RX], m["u"][0][0, RX:nx - RX]))
        return out
    finally:
        oracle.set_threads(prev)


def l1_against_exact(steps, rho, u):
    r = oracle.Lattice(2, 33).r
    xs = np.arange(1000, dtype=float)
    re, ue, _ = riemann.sample(LEFT, RIGHT, G, (xs - 499.5) * r / steps)
    return np.abs(rho - re).sum() / re.sum(), np.abs(u - ue).sum() / np.abs(ue).sum()


def test_open_ends_keep_a_uniform_state():
    """Zero-gradient ends continue a uniform moving equilibrium exactly."""
    for Q in (33, 37):
        nx, ny = 24, 9
        sim = oracle.Sim(2, Q, 3, 0.71, 0.8, (nx, ny))
        sim.init(np.full((ny, nx), 1.2), np.stack([np.full((ny, nx), 0.1), np.full((ny, nx), -0.05)]),
                 np.full((ny, nx), 1.05))
        sim.set_open_x(True)
        sim.step(30)
        m = sim.moments()
        assert np.max(np.abs(m["rho"] / 1.2 - 1)) < 1e-13 and np.max(np.abs(m["T"] / 1.05 - 1)) < 1e-13
        assert np.max(np.abs(m["u"][0] - 0.1)) < 1e-13 and np.max(np.abs(m["u"][1] + 0.05)) < 1e-13


def test_open_ends_let_the_waves_leave():
    """The whole 1000-cell tube with open ends follows the exact solution of
    the infinite tube at t ~ 0.15 (174 steps) and still after the shock
    (~290 steps) and the rarefaction head (~470 steps) have reached the
    ends (500 steps): little is reflected.  A periodic tube of the same
    length does not (its wrap is a second interface)."""
    for steps, rho, u in open_tube([174, 500]):
        e_rho, e_u = l1_against_exact(steps, rho, u)
        print(f"open tube {steps} steps: L1 rho {e_rho:.3e} u {e_u:.3e}")
        assert e_rho < 0.02 and e_u < 0.04, (steps, e_rho, e_u)
    (steps, rho, u), = open_tube([500], open_x=False)
    e_rho, e_u = l1_against_exact(steps, rho, u)
    assert e_rho > 0.3 and e_u > 0.5
