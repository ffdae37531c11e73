"""Pins of the oracle's 1D quadrature matrices (Sec. 2.5 1D integrals)."""
import numpy as np
import pytest
from scipy.special import erf

from oracle.assemble import Dim1D


def _dim(n=12, s=2, p=2, n_gauss=5, L=1.0, seed=0):
    x = np.linspace(0.0, L, n)
    rng = np.random.Generator(np.random.PCG64(seed))
    x[1:-1] += rng.uniform(-0.2, 0.2, n - 2) * L / (n - 1)
    return Dim1D(x, s, 20.0, p, n_gauss)


@pytest.mark.parametrize("s,p", [(2, 2), (1, 1), (3, 3), (2, 1)])
def test_moments_of_polynomials(s, p):
    D = _dim(s=s, p=p, L=1.7)
    L = D.nodes[-1]
    Mm, K, G = D.matrix("mass").toarray(), D.matrix("stiff").toarray(), D.matrix("ddt").toarray()
    x = D.nodes
    for q in range(p + 1):
        for r in range(p + 1):
            assert abs(x ** q @ Mm @ x ** r - L ** (q + r + 1) / (q + r + 1)) < 1e-12
            if q > 0 and r > 0:
                exact = q * r * L ** (q + r - 1) / (q + r - 1)
                assert abs(x ** q @ K @ x ** r - exact) < 1e-10
    assert abs(np.ones_like(x) @ G @ x - L) < 1e-12
    assert np.abs(K @ np.ones_like(x)).max() < 1e-10


def test_time_derivative_integration_by_parts():
    D = _dim(n=15)
    G = D.matrix("ddt").toarray()
    E = np.zeros_like(G)
    E[-1, -1] = 1.0
    E[0, 0] = -1.0
    assert np.abs(G + G.T - E).max() < 1e-12


def test_symmetric_and_definite():
    D = _dim(n=14)
    Mm, K = D.matrix("mass").toarray(), D.matrix("stiff").toarray()
    assert np.abs(Mm - Mm.T).max() < 1e-15 and np.abs(K - K.T).max() < 1e-12
    assert np.linalg.eigvalsh(Mm).min() > 0
    assert np.linalg.eigvalsh(K[1:, 1:]).min() > 0


def test_quadrature_exact_for_polynomial_basis():
    # with a >= 2(s+1) each Ntilde is a polynomial of degree <= 4 per element, so
    # 5-point Gauss integrates mass / stiffness / time-derivative exactly
    A, B = _dim(n_gauss=5), _dim(n_gauss=8)
    for kind in ("mass", "stiff", "ddt"):
        assert np.abs((A.matrix(kind) - B.matrix(kind)).toarray()).max() < 1e-11
    lin = lambda x: 1.0 + 2.0 * x
    Wa, Wb = A.matrix("wmass", coef=lin), B.matrix("wmass", coef=lin)
    assert np.abs((Wa - Wb).toarray()).max() < 1e-12


def test_s0_textbook_linear_elements():
    n = 9
    D = Dim1D(np.linspace(0, 1, n), 0, 3.0, 0, 2)
    h = 1.0 / (n - 1)
    K, Mm = D.matrix("stiff").toarray(), D.matrix("mass").toarray()
    for i in range(1, n - 1):
        assert np.allclose(K[i, i - 1:i + 2], np.array([-1, 2, -1]) / h, atol=1e-12)
        assert np.allclose(Mm[i, i - 1:i + 2], np.array([1, 4, 1]) * h / 6, atol=1e-15)


def test_band_half_width():
    D = _dim(n=20, s=2)
    A = D.matrix("stiff").tocoo()
    assert np.max(np.abs(A.row - A.col)) == 2 * 2 + 1


def test_gaussian_load_total():
    # 1^T F = int f (partition of unity), compared with the closed form via erf
    D = Dim1D(np.linspace(0, 1, 200), 2, 20.0, 2, 5)
    c, r = 0.37, 0.05
    F = D.load(lambda x: np.exp(-2 * (x - c) ** 2 / r ** 2))
    s2 = np.sqrt(2.0) / r
    exact = np.sqrt(np.pi) / (2 * s2) * (erf(s2 * (1 - c)) - erf(s2 * (0 - c)))
    assert abs(F.sum() - exact) < 1e-9 * exact


@pytest.mark.parametrize("s,p", [(2, 2), (1, 1), (3, 3)])
def test_weighted_mass_moments_with_linear_coefficient(s, p):
    # for a coefficient c(x) = alpha + beta x and q, r <= p the reproducing
    # property makes (x^q)^T W^c x^r the exact integral of c(x) x^(q+r) over the
    # domain: a dropped, squared or misplaced coefficient changes these values
    D = _dim(n=13, s=s, p=p, L=1.3, seed=3)
    a0, b0 = D.nodes[0], D.nodes[-1]
    alpha, beta = 0.7, -1.9
    W = D.matrix("wmass", coef=lambda x: alpha + beta * x).toarray()
    x = D.nodes
    for q in range(p + 1):
        for r in range(p + 1):
            k = q + r
            exact = alpha * (b0 ** (k + 1) - a0 ** (k + 1)) / (k + 1) + beta * (b0 ** (k + 2) - a0 ** (k + 2)) / (k + 2)
            assert abs(x ** q @ W @ x ** r - exact) < 1e-12 * max(1.0, abs(exact))
    # a constant coefficient gives c times the mass matrix, entry by entry
    Wc = D.matrix("wmass", coef=lambda x: 2.5 * np.ones_like(x)).toarray()
    assert np.abs(Wc - 2.5 * D.matrix("mass").toarray()).max() < 1e-15
    # coefficient values given at the Gauss points are the callable's values there
    Wv = D.matrix("wmass", coef=alpha + beta * D.xg).toarray()
    assert np.abs(Wv - W).max() == 0.0


@pytest.mark.parametrize("s,p", [(2, 2), (1, 1), (3, 3)])
def test_weighted_stiffness_and_product_derivative_moments(s, p):
    # c(x) = alpha + beta x: (x^q)^T W_K x^r = q r int c x^(q+r-2), and
    # (x^q)^T W_G x^r = int x^q (c x^r)' exactly for q, r <= p; with q = 0 the
    # latter is c x^r between the domain ends (integration by parts pins the
    # product rule, not only the sum of its two parts)
    D = _dim(n=13, s=s, p=p, L=1.3, seed=5)
    a0, b0 = D.nodes[0], D.nodes[-1]
    alpha, beta = 0.7, -1.9
    c = lambda x: alpha + beta * x
    WK = D.matrix("wstiff", coef=c).toarray()
    WG = D.matrix("wddt", coef=c, dcoef=lambda x: beta * np.ones_like(x)).toarray()
    x = D.nodes
    P = lambda k: (b0 ** k - a0 ** k) / k   # int x^(k-1)
    for q in range(p + 1):
        for r in range(p + 1):
            if q > 0 and r > 0:
                k = q + r - 2
                exact = q * r * (alpha * P(k + 1) + beta * P(k + 2))
                assert abs(x ** q @ WK @ x ** r - exact) < 1e-10 * max(1.0, abs(exact))
            # int x^q (alpha x^r + beta x^(r+1))' = int x^q (alpha r x^(r-1) + beta (r+1) x^r)
            exact = (alpha * r * P(q + r) if r > 0 else 0.0) + beta * (r + 1) * P(q + r + 1)
            assert abs(x ** q @ WG @ x ** r - exact) < 1e-11 * max(1.0, abs(exact))
        ends = c(b0) * b0 ** q - c(a0) * a0 ** q
        assert abs(np.ones_like(x) @ WG @ x ** q - ends) < 1e-11 * max(1.0, abs(ends))
    # a constant coefficient gives c times the plain kinds
    Kc = D.matrix("wstiff", coef=lambda x: 2.5 * np.ones_like(x)).toarray()
    Gc = D.matrix("wddt", coef=lambda x: 2.5 * np.ones_like(x), dcoef=lambda x: np.zeros_like(x)).toarray()
    assert np.abs(Kc - 2.5 * D.matrix("stiff").toarray()).max() < 1e-12
    assert np.abs(Gc - 2.5 * D.matrix("ddt").toarray()).max() < 1e-14
