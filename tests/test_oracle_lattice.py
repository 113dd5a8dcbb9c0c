"""Pins of the oracle's lattice solve against the paper's printed tables and
against brute-force quadrature exactness (CPU only)."""
import itertools
import math

import numpy as np
import pytest

import oracle
from conftest import read_table


def gauss_moment_1d(e):
    """E[x^e] for x ~ N(0, 1): 0 for odd e, (e-1)!! for even e."""
    if e % 2:
        return 0.0
    return float(math.prod(range(e - 1, 0, -2))) if e > 0 else 1.0


def lattice_moment(L, exps):
    xi = L.xi
    return float(np.sum(L.w * np.prod([xi[:, d] ** exps[d] for d in range(L.D)], axis=0)))


@pytest.mark.parametrize("D,Q,deg", [(2, 37, 9), (2, 33, 9), (3, 39, 7)])
def test_quadrature_exact_to_degree(D, Q, deg):
    """Every monomial of total degree <= deg (odd ones included) integrates
    exactly against the unit Gaussian weight -- the defining property of the
    Hermite quadrature the lattices are built on (Section VI.A)."""
    L = oracle.Lattice(D, Q)
    for total in range(deg + 1):
        for exps in itertools.product(range(total + 1), repeat=D):
            if sum(exps) != total:
                continue
            want = math.prod(gauss_moment_1d(e) for e in exps)
            got = lattice_moment(L, exps)
            assert abs(got - want) <= 1e-13 * max(1.0, want), (exps, got, want)


@pytest.mark.parametrize("D,Q,deg", [(2, 37, 9), (2, 33, 9), (3, 39, 7)])
def test_quadrature_degree_is_tight(D, Q, deg):
    """The next even degree is not exact (the solve did not degenerate)."""
    L = oracle.Lattice(D, Q)
    e = deg + 1
    exps = (e,) + (0,) * (D - 1)
    assert abs(lattice_moment(L, exps) - gauss_moment_1d(e)) > 1e-3


def _shell_key(c):
    return tuple(sorted((abs(int(v)) for v in c), reverse=True))


@pytest.mark.parametrize("fname,D,Q,wtol,rtol", [("table1_d2q37.txt", 2, 37, 6e-9, 1e-8),
                                                   ("table2_d2q33.txt", 2, 33, 1.0e-6, 1e-6)])
def test_matches_printed_table(fname, D, Q, wtol, rtol):
    """Solved weights and r agree with Table I / Table II to the printed
    precision (D2Q37 9 digits: the small-weight entries of Table I carry
    about 3e-9 absolute rounding; D2Q33: 6 digits)."""
    r_print, rows = read_table(fname)
    L = oracle.Lattice(D, Q)
    assert abs(L.r - r_print) <= rtol
    keys = [_shell_key(c) for c in L.c]
    for k, a, b, w in rows:
        key = (max(a, b), min(a, b))
        members = [i for i, kk in enumerate(keys) if kk == key]
        assert len(members) == k, (key, len(members), k)
        for i in members:
            assert abs(L.w[i] - w) <= wtol, (key, L.w[i], w)


def test_d3q39_rational_weights():
    """D3Q39 (not in the paper) solves to rational weights and r^2 = 3/2."""
    L = oracle.Lattice(3, 39)
    want = {(0, 0, 0): 1 / 12, (1, 0, 0): 1 / 12, (1, 1, 1): 1 / 27, (2, 0, 0): 2 / 135, (2, 2, 0): 1 / 432,
            (3, 0, 0): 1 / 1620}
    for i, c in enumerate(L.c):
        assert abs(L.w[i] - want[_shell_key(c)]) < 1e-15
    assert abs(L.r ** 2 - 1.5) < 1e-15


@pytest.mark.parametrize("D,Q,reach", [(2, 37, 3), (2, 33, 4), (3, 39, 3)])
def test_velocity_set_structure(D, Q, reach):
    L = oracle.Lattice(D, Q)
    assert L.c.shape == (Q, D)
    assert len({tuple(c) for c in L.c}) == Q
    for i in range(Q):
        assert np.array_equal(L.c[L.opp[i]], -L.c[i])
    assert np.abs(L.c).max() == reach
    assert abs(L.w.sum() - 1.0) < 1e-15
