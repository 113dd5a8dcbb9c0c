"""Exact solution of the one-dimensional Riemann problem of an ideal gas
(the reference for the shock-tube validation of Sec. VI.B of the paper).

TEST INFRASTRUCTURE ONLY (part of the oracle).

Two constant states (rho, u, p) meet at x = 0 at t = 0.  The solution is
self-similar in s = x/t: a left wave (rarefaction or shock), a contact, and
a right wave.  The star-region pressure p* solves f_L(p*) + f_R(p*) + u_R -
u_L = 0, where for each side K with sound speed c_K = sqrt(gamma p_K/rho_K)

  shock (p* > p_K):        f_K = (p* - p_K) sqrt(A_K / (p* + B_K)),
                           A_K = 2/((gamma+1) rho_K), B_K = (gamma-1)/(gamma+1) p_K
  rarefaction (p* <= p_K): f_K = 2 c_K/(gamma-1) ((p*/p_K)^((gamma-1)/(2 gamma)) - 1)

(the Rankine-Hugoniot and isentropic relations written as functions of the
pressure), solved by Newton's method; u* = (u_L + u_R + f_R - f_L)/2.
"""
from __future__ import annotations

import numpy as np


def _f(p, rho, pk, g):
    c = np.sqrt(g * pk / rho)
    if p > pk:
        A = 2.0 / ((g + 1) * rho)
        B = (g - 1) / (g + 1) * pk
        f = (p - pk) * np.sqrt(A / (p + B))
        df = np.sqrt(A / (B + p)) * (1 - (p - pk) / (2 * (B + p)))
    else:
        f = 2 * c / (g - 1) * ((p / pk) ** ((g - 1) / (2 * g)) - 1)
        df = 1 / (rho * c) * (p / pk) ** (-(g + 1) / (2 * g))
    return f, df


def star_state(left, right, gamma):
    """(p*, u*) of the Riemann problem with states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    p = 0.5 * (pl + pr)
    for _ in range(100):
        fl, dfl = _f(p, rl, pl, gamma)
        fr, dfr = _f(p, rr, pr, gamma)
        dp = (fl + fr + ur - ul) / (dfl + dfr)
        p = max(p - dp, 1e-14)
        if abs(dp) < 1e-15 * p:
            break
    fl, _ = _f(p, rl, pl, gamma)
    fr, _ = _f(p, rr, pr, gamma)
    return p, 0.5 * (ul + ur + fr - fl)


def sample(left, right, gamma, s):
    """(rho, u, p) at the similarity coordinates s = x/t (array)."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(left, right, gamma)
    g = gamma
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    s = np.asarray(s, dtype=float)
    rho, u, p = np.empty_like(s), np.empty_like(s), np.empty_like(s)
    for k, x in enumerate(s):
        if x <= us:                              # left of the contact
            if ps > pl:                          # left shock
                sl = ul - cl * np.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                if x <= sl:
                    rho[k], u[k], p[k] = rl, ul, pl
                else:
                    r = rl * (ps / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pl + 1)
                    rho[k], u[k], p[k] = r, us, ps
            else:                                # left rarefaction
                csl = cl * (ps / pl) ** ((g - 1) / (2 * g))
                if x <= ul - cl:
                    rho[k], u[k], p[k] = rl, ul, pl
                elif x >= us - csl:
                    rho[k], u[k], p[k] = rl * (ps / pl) ** (1 / g), us, ps
                else:
                    uu = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + x)
                    c = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - x))
                    r = rl * (c / cl) ** (2 / (g - 1))
                    rho[k], u[k], p[k] = r, uu, pl * (c / cl) ** (2 * g / (g - 1))
        else:                                    # right of the contact
            if ps > pr:                          # right shock
                sr = ur + cr * np.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                if x >= sr:
                    rho[k], u[k], p[k] = rr, ur, pr
                else:
                    r = rr * (ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1)
                    rho[k], u[k], p[k] = r, us, ps
            else:                                # right rarefaction
                csr = cr * (ps / pr) ** ((g - 1) / (2 * g))
                if x >= ur + cr:
                    rho[k], u[k], p[k] = rr, ur, pr
                elif x <= us + csr:
                    rho[k], u[k], p[k] = rr * (ps / pr) ** (1 / g), us, ps
                else:
                    uu = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + x)
                    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - x))
                    r = rr * (c / cr) ** (2 / (g - 1))
                    rho[k], u[k], p[k] = r, uu, pr * (c / cr) ** (2 * g / (g - 1))
    return rho, u, p
