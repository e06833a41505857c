"""Pins of the oracle's basis and quadrature against mathematics fixed
independently of the oracle (library routines, the paper's Rodrigues formula,
closed-form monomial integrals, direct evaluation of the collapsed formula)."""
from math import comb, factorial

import numpy as np
import pytest
from numpy.polynomial import polynomial as P1
from scipy.special import eval_jacobi

from oracle.basis import Dubiner, jacobi, modes, tet_quadrature, tri_quadrature


@pytest.mark.parametrize("n", range(0, 8))
@pytest.mark.parametrize("ab", [(0, 0), (1, 0), (3, 0), (5, 0), (2, 1), (8, 0)])
def test_jacobi_matches_scipy(n, ab):
    w = np.linspace(-1, 1, 41)
    np.testing.assert_allclose(jacobi(n, *ab, w), eval_jacobi(n, ab[0], ab[1], w),
                               rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n", range(0, 6))
@pytest.mark.parametrize("a", [0, 1, 3, 6])
def test_jacobi_matches_rodrigues(n, a):
    """Generating formula of Sec. II (Rodrigues) with integer alpha=a, beta=0:
    P_n = (-1)^n/(2^n n!) (1-w)^-a d^n/dw^n [(1-w)^(a+n) (1+w)^n]."""
    from fractions import Fraction
    # exact integer coefficients of (1-w)^(a+n) (1+w)^n, then the n-th derivative
    c = [1]
    for fac in [[1, -1]] * (a + n) + [[1, 1]] * n:
        out = [0] * (len(c) + 1)
        for i, ci in enumerate(c):
            out[i] += ci * fac[0]
            out[i + 1] += ci * fac[1]
        c = out
    for _ in range(n):
        c = [i * ci for i, ci in enumerate(c)][1:]
    ws = [Fraction(k, 20) for k in range(-19, 20, 2)]
    vals = []
    for w in ws:
        poly = sum(Fraction(ci) * w ** i for i, ci in enumerate(c))
        vals.append(float(Fraction((-1) ** n, 2 ** n * factorial(n)) * poly / (1 - w) ** a))
    np.testing.assert_allclose(jacobi(n, a, 0, np.array([float(w) for w in ws])), vals,
                               rtol=1e-13, atol=1e-13)


def _dirichlet(a, b, c):
    # int_T x^a y^b z^c = a! b! c! / (a+b+c+3)!
    return factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 3)


@pytest.mark.parametrize("q", [2, 3, 4, 5])
def test_tet_quadrature_exact_on_monomials(q):
    pts, w = tet_quadrature(q)
    assert abs(w.sum() - 1.0 / 6.0) < 1e-15
    for a in range(2 * q):
        for b in range(2 * q - a):
            for c in range(2 * q - a - b):
                num = np.sum(w * pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c)
                assert abs(num - _dirichlet(a, b, c)) < 1e-15, (a, b, c)


@pytest.mark.parametrize("q", [2, 3, 5])
def test_tri_quadrature_exact_on_monomials(q):
    pts, w = tri_quadrature(q)
    for a in range(2 * q):
        for b in range(2 * q - a):
            exact = factorial(a) * factorial(b) / factorial(a + b + 2)
            num = np.sum(w * pts[:, 0] ** a * pts[:, 1] ** b)
            assert abs(num - exact) < 1e-15


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4])
def test_mode_count(p):
    """N = C(p+3, 3) (Sec. II)."""
    assert len(modes(p)) == comb(p + 3, 3)
    assert Dubiner(p).N == comb(p + 3, 3)


def _collapsed_direct(i, j, k, x, y, z):
    """The corrected collapsed formula evaluated directly with scipy's Jacobi."""
    nrm = np.sqrt((2 * i + 1) * (2 * i + 2 * j + 2) * (2 * i + 2 * j + 2 * k + 3))
    return (nrm * eval_jacobi(i, 0, 0, 2 * z / (1 - x - y) - 1) * (1 - x - y) ** i
            * eval_jacobi(j, 2 * i + 1, 0, 2 * y / (1 - x) - 1) * (1 - x) ** j
            * eval_jacobi(k, 2 * i + 2 * j + 2, 0, 2 * x - 1))


@pytest.mark.parametrize("p", [2, 3, 4])
def test_monomial_expansion_matches_collapsed_formula(p):
    rng = np.random.default_rng(7)
    lam = rng.dirichlet(np.ones(4), size=50)  # strictly interior points
    pts = lam[:, 1:]
    B = Dubiner(p)
    V = B.eval(pts)
    for m, (i, j, k) in enumerate(B.modes):
        ref = _collapsed_direct(i, j, k, pts[:, 0], pts[:, 1], pts[:, 2])
        np.testing.assert_allclose(V[:, m], ref, rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("p", [2, 3, 4])
def test_orthonormal_exact_integration(p):
    """Gram matrix = I (eq. ortho_cond), by exact monomial integration."""
    B = Dubiner(p)
    ex = B.exps
    M = np.array([[_dirichlet(a1 + a2, b1 + b2, c1 + c2) for (a2, b2, c2) in ex]
                  for (a1, b1, c1) in ex])
    G = B.coef @ M @ B.coef.T
    # monomial coefficients grow with p; allow their cancellation error
    np.testing.assert_allclose(G, np.eye(B.N), atol=1e-16 * np.abs(B.coef).max() ** 2)
    assert abs(B.eval(np.zeros((1, 3)))[0, 0] - np.sqrt(6.0)) < 1e-14


@pytest.mark.parametrize("p", [2, 3])
def test_gradient_matches_finite_differences(p):
    B = Dubiner(p)
    rng = np.random.default_rng(3)
    pts = rng.dirichlet(np.ones(4), size=20)[:, 1:]
    g = B.grad(pts)
    h = 1e-6
    for ax in range(3):
        d = np.zeros(3)
        d[ax] = h
        fd = (B.eval(pts + d) - B.eval(pts - d)) / (2 * h)
        np.testing.assert_allclose(g[:, ax, :], fd, rtol=1e-7, atol=1e-7)


def test_printed_formula_is_not_orthogonal():
    """Documents the reading: the formula as typeset (no (1-x)^j factor, third
    Jacobi parameter (2i+1,0)) is not an orthogonal set."""
    pts, w = tet_quadrature(8)
    x, y, z = pts.T

    def printed(i, j, k):
        return (eval_jacobi(i, 0, 0, 2 * z / (1 - x - y) - 1) * (1 - x - y) ** i
                * eval_jacobi(j, 2 * i + 1, 0, 2 * y / (1 - x) - 1)
                * eval_jacobi(k, 2 * i + 1, 0, 2 * x - 1))

    F = np.array([printed(*m) for m in modes(2)])
    G = (F * w) @ F.T
    off = G - np.diag(np.diag(G))
    assert np.abs(off).max() > 1e-3
