"""Pins of the oracle's Hermite tensors, general-term coefficients and
discrete target against independent constructions (CPU only):

* one-dimensional probabilists' Hermite polynomials from numpy,
* brute-force Gauss-Hermite quadrature of the continuous Gaussian,
* the separable closed form for a diagonal covariance,
* the second-order contraction printed in Appendix B.
"""
import itertools
import math

import numpy as np
import pytest
from numpy.polynomial import hermite_e as He

import oracle


def he(m, x):
    return He.hermeval(x, [0] * m + [1])


def hermite_by_products(n, xi):
    """H^(n)_{i1..in}(xi) = prod_d He_{m_d}(xi_d), m_d = how many indices equal d."""
    D = len(xi)
    out = np.zeros((D,) * n)
    for idx in itertools.product(range(D), repeat=n):
        out[idx] = math.prod(he(idx.count(d), xi[d]) for d in range(D))
    return out


def gauss_expectation(u, Lam, fn, K=12):
    """E[fn(xi)] for xi ~ N(u, Lam) by a K^D tensor Gauss-Hermite rule
    (exact for polynomials of degree <= 2K-1)."""
    D = len(u)
    x, w = He.hermegauss(K)
    w = w / w.sum()
    Lc = np.linalg.cholesky(Lam)
    tot = 0.0
    for ids in itertools.product(range(K), repeat=D):
        eta = x[list(ids)]
        tot += np.prod(w[list(ids)]) * fn(u + Lc @ eta)
    return tot


def random_spd(D, rng, lo=0.6, hi=1.5):
    Qm, _ = np.linalg.qr(rng.standard_normal((D, D)))
    return Qm @ np.diag(rng.uniform(lo, hi, D)) @ Qm.T


@pytest.mark.parametrize("D", [2, 3])
@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5, 6])
def test_hermite_tensor_is_product_of_1d(D, n):
    rng = np.random.default_rng(10 * D + n)
    for _ in range(3):
        xi = rng.standard_normal(D) * 1.5
        np.testing.assert_allclose(oracle.hermite(n, xi), hermite_by_products(n, xi), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("D", [2, 3])
@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5, 6])
def test_general_term_matches_quadrature(D, n):
    """a^(n) = (1/rho) int H^(n)(xi) G dxi (Eq. HermiteCo) for a random
    anisotropic Gaussian, integrated by brute force."""
    rng = np.random.default_rng(100 + 10 * D + n)
    u = rng.uniform(-0.4, 0.4, D)
    Lam = random_spd(D, rng)
    a = oracle.coeff(n, u, Lam - np.eye(D))
    K = 8 if D == 3 else 12
    for idx in itertools.product(range(D), repeat=n):
        want = gauss_expectation(u, Lam, lambda xi: math.prod(he(idx.count(d), xi[d]) for d in range(D)), K=K)
        assert abs(a[idx] - want) <= 1e-12 * max(1.0, abs(want)), (idx, a[idx], want)


def h_sep(m, mu, a):
    """1D Hermite coefficient of N(mu, 1 + a): sum_k m!/(k!(m-2k)!2^k) a^k mu^(m-2k)."""
    return sum(math.factorial(m) / (math.factorial(k) * math.factorial(m - 2 * k) * 2 ** k) * a ** k * mu ** (m - 2 * k)
               for k in range(m // 2 + 1))


@pytest.mark.parametrize("D", [2, 3])
def test_diagonal_covariance_closed_form(D):
    rng = np.random.default_rng(7 + D)
    u = rng.uniform(-0.5, 0.5, D)
    lam = rng.uniform(0.5, 1.6, D)
    A = np.diag(lam - 1.0)
    for n in range(7):
        a = oracle.coeff(n, u, A)
        for idx in itertools.product(range(D), repeat=n):
            want = math.prod(h_sep(idx.count(d), u[d], lam[d] - 1.0) for d in range(D))
            assert abs(a[idx] - want) < 1e-13 * max(1.0, abs(want))


def test_appendix_b_second_order_contraction():
    """a^(2).H^(2) = Lambda_ij xi_i xi_j - Lambda_ii - xi^2 + D + (u.xi)^2 - u^2
    (Appendix B, second line)."""
    rng = np.random.default_rng(3)
    for D in (2, 3):
        for _ in range(5):
            u = rng.uniform(-0.5, 0.5, D)
            Lam = random_spd(D, rng)
            xi = rng.standard_normal(D) * 2
            lhs = float(np.sum(oracle.coeff(2, u, Lam - np.eye(D)) * oracle.hermite(2, xi)))
            rhs = xi @ Lam @ xi - np.trace(Lam) - xi @ xi + D + (u @ xi) ** 2 - u @ u
            assert abs(lhs - rhs) < 1e-13


def _moment_tensor_from_pops(L, G, m):
    xi = L.xi
    out = np.zeros((L.D,) * m)
    for idx in itertools.product(range(L.D), repeat=m):
        out[idx] = np.sum(G * np.prod([xi[:, d] for d in idx], axis=0)) if m else np.sum(G)
    return out


@pytest.mark.parametrize("D,Q,mmax", [(2, 37, 4), (2, 33, 4), (3, 39, 3)])
def test_target_moments_equal_gaussian_moments(D, Q, mmax):
    """sum_i G_i xi_i^m = rho E_{N(u, Lambda)}[xi^m] for every m up to the
    order the truncation and the quadrature degree guarantee (4 in 2D with a
    degree-9 rule, 3 for D3Q39's degree-7 rule)."""
    L = oracle.Lattice(D, Q)
    rng = np.random.default_rng(D * 100 + Q)
    for _ in range(3):
        rho = rng.uniform(0.8, 1.3)
        u = rng.uniform(-0.3, 0.3, D)
        Lam = random_spd(D, rng, 0.7, 1.3)
        G = oracle.equilibrium(D, Q, rho, u, Lam - np.eye(D))
        K = 6
        for m in range(mmax + 1):
            got = _moment_tensor_from_pops(L, G, m)
            for idx in itertools.product(range(D), repeat=m):
                want = rho * gauss_expectation(u, Lam, lambda xi: math.prod(xi[d] for d in idx), K=K)
                g = got[idx] if m else got
                assert abs(g - want) < 1e-12, (m, idx, g, want)


def test_d2q37_fifth_moment_differs_from_gaussian():
    """The order-4 truncation does not carry the Gaussian's fifth moment:
    the mmax above is the right bound, not a loose one."""
    L = oracle.Lattice(2, 37)
    u = np.array([0.3, -0.2])
    Lam = np.array([[1.2, 0.1], [0.1, 0.9]])
    G = oracle.equilibrium(2, 37, 1.0, u, Lam - np.eye(2))
    got = np.sum(G * L.xi[:, 0] ** 5)
    want = gauss_expectation(u, Lam, lambda xi: xi[0] ** 5)
    assert abs(got - want) > 1e-4


@pytest.mark.parametrize("D,Q", [(2, 37), (3, 39), (2, 33)])
def test_isotropic_target_is_separable_maxwellian(D, Q):
    """Lambda = T delta (the BGK case) and any diagonal Lambda: G_i equals
    w_i rho sum_{|m|<=4} prod_d h_{m_d}(u_d, lambda_d - 1) He_{m_d}(xi_d)/m_d!."""
    L = oracle.Lattice(D, Q)
    rng = np.random.default_rng(11)
    for iso in (True, False):
        rho = 1.1
        u = rng.uniform(-0.3, 0.3, D)
        lam = np.full(D, 1.07) if iso else rng.uniform(0.8, 1.2, D)
        G = oracle.equilibrium(D, Q, rho, u, np.diag(lam - 1.0))
        want = np.zeros(Q)
        for i in range(Q):
            s = 0.0
            for ms in itertools.product(range(5), repeat=D):
                if sum(ms) > 4:
                    continue
                s += math.prod(h_sep(ms[d], u[d], lam[d] - 1.0) * he(ms[d], L.xi[i, d]) / math.factorial(ms[d])
                               for d in range(D))
            want[i] = L.w[i] * rho * s
        np.testing.assert_allclose(G, want, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("D,Q", [(2, 37), (3, 39)])
def test_rest_state_target_is_weights(D, Q):
    L = oracle.Lattice(D, Q)
    G = oracle.equilibrium(D, Q, 1.7, np.zeros(D), np.zeros((D, D)))
    np.testing.assert_allclose(G, 1.7 * L.w, rtol=1e-14)
