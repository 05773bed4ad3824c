"""Pins of the oracle's reference elements (Sec. 1.2): orthonormality under (1/|T0|) int, phi_1 == 1,
closed forms of the low modes, and exactness of the quadrature rules.  The checks use an
independent high-order rule (tensor / collapsed Gauss-Legendre from numpy), never the oracle's."""
import math

import numpy as np
import pytest

import oracle as O


def hi_rule(kind, n=10):
    """Independent quadrature: points (P x dim) and weights normalised by |T0|."""
    x, w = np.polynomial.legendre.leggauss(n)
    if kind == O.LINE:
        return x[:, None], w / 2.0
    if kind == O.QUAD:
        X, Y = np.meshgrid(x, x, indexing="ij")
        W = np.outer(w, w)
        return np.stack([X.ravel(), Y.ravel()], 1), W.ravel() / 4.0
    # collapsed (Duffy) rule on the triangle (0,0),(1,0),(0,1): xi = u, eta = (1-u) v
    u = 0.5 * (x + 1)
    wu = 0.5 * w
    U, Vv = np.meshgrid(u, u, indexing="ij")
    W = np.outer(wu, wu) * (1 - U)
    return np.stack([U.ravel(), ((1 - U) * Vv).ravel()], 1), 2.0 * W.ravel()


@pytest.mark.parametrize("kind", [O.LINE, O.QUAD, O.TRI])
def test_basis_orthonormal(kind):
    R = O.RefElem(kind)
    pts, w = hi_rule(kind)
    Phi = np.array([[R.phi(l, p) for p in pts] for l in range(R.ML)])
    G = (Phi * w) @ Phi.T
    assert np.allclose(G, np.eye(R.ML), atol=1e-13)
    assert np.allclose(Phi[0], 1.0, atol=1e-15)


def test_basis_closed_forms():
    L = O.RefElem(O.LINE)
    for xi in [-0.9, -0.2, 0.35, 1.0]:
        assert L.phi(1, [xi]) == pytest.approx(math.sqrt(3) * xi, abs=1e-14)
        assert L.phi(2, [xi]) == pytest.approx(math.sqrt(5) / 2 * (3 * xi * xi - 1), abs=1e-14)
    T = O.RefElem(O.TRI)
    for xi, eta in [(0.1, 0.2), (0.5, 0.25), (0.0, 1.0), (1 / 3, 1 / 3)]:
        # Gram-Schmidt of 1, xi, eta by hand: sqrt(2)(3 xi - 1) and sqrt(6)(xi + 2 eta - 1)
        assert T.phi(1, [xi, eta]) == pytest.approx(math.sqrt(2) * (3 * xi - 1), abs=1e-13)
        assert T.phi(2, [xi, eta]) == pytest.approx(math.sqrt(6) * (xi + 2 * eta - 1), abs=1e-13)
    Qd = O.RefElem(O.QUAD)
    for xi, eta in [(0.1, -0.7), (0.9, 0.3)]:
        p1 = lambda s: math.sqrt(3) * s
        p2 = lambda s: math.sqrt(5) / 2 * (3 * s * s - 1)
        expect = [1, p1(xi), p1(eta), p2(xi), p1(xi) * p1(eta), p2(eta), p2(xi) * p1(eta), p1(xi) * p2(eta), p2(xi) * p2(eta)]
        got = [Qd.phi(l, [xi, eta]) for l in range(9)]
        assert np.allclose(got, expect, atol=1e-13)


@pytest.mark.parametrize("kind", [O.LINE, O.QUAD, O.TRI])
def test_basis_derivatives_match_differences(kind):
    R = O.RefElem(kind)
    rng = np.random.default_rng(1)
    h = 1e-5
    for _ in range(5):
        p = rng.uniform(0.05, 0.4, R.dim)
        for l in range(R.ML):
            for a in range(R.dim):
                e = np.zeros(R.dim)
                e[a] = h
                fd = (R.phi(l, p + e) - R.phi(l, p - e)) / (2 * h)
                got = R.phi(l, p, *(1, 0) if a == 0 else (0, 1))
                assert got == pytest.approx(fd, abs=1e-7)
                fd2 = (R.phi(l, p + e) - 2 * R.phi(l, p) + R.phi(l, p - e)) / h**2
                got2 = R.phi(l, p, *(2, 0) if a == 0 else (0, 2))
                assert got2 == pytest.approx(fd2, abs=1e-3)


def exact_moment(kind, a, b):
    if kind == O.LINE:
        return 0.0 if a % 2 else 1.0 / (a + 1)
    if kind == O.QUAD:
        f = lambda n: 0.0 if n % 2 else 1.0 / (n + 1)
        return f(a) * f(b)
    return 2.0 * math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)


@pytest.mark.parametrize("kind,deg", [(O.LINE, 5), (O.QUAD, 5), (O.TRI, 5)])
def test_interior_rule_exactness(kind, deg):
    R = O.RefElem(kind)
    assert R.w_int.sum() == pytest.approx(1.0, abs=1e-15)
    for a in range(deg + 1):
        for b in range(deg + 1):
            if R.dim == 1 and b > 0:
                continue
            if kind == O.TRI and a + b > deg:
                continue
            x = R.xi_int[:, 0]
            y = R.xi_int[:, 1] if R.dim == 2 else np.ones_like(x)
            got = np.sum(R.w_int * x**a * y**b)
            assert got == pytest.approx(exact_moment(kind, a, b), abs=1e-14), (a, b)
    if kind == O.TRI:  # not exact at degree 6 (it is a degree-5 rule)
        x, y = R.xi_int[:, 0], R.xi_int[:, 1]
        assert abs(np.sum(R.w_int * x**6) - exact_moment(kind, 6, 0)) > 1e-8


@pytest.mark.parametrize("kind", [O.QUAD, O.TRI])
def test_edge_points_on_edges(kind):
    R = O.RefElem(kind)
    verts = {O.QUAD: [(-1, -1), (1, -1), (1, 1), (-1, 1)], O.TRI: [(0, 0), (1, 0), (0, 1)]}[kind]
    assert R.om_edge.sum() == pytest.approx(2.0, abs=1e-15)
    s = np.array([-math.sqrt(0.6), 0.0, math.sqrt(0.6)])
    for k in range(R.K):
        a, b = np.array(verts[k]), np.array(verts[(k + 1) % len(verts)])
        for j in range(R.NQE):
            expect = a + 0.5 * (1 + s[j]) * (b - a)
            assert np.allclose(R.xi_edge[k, j], expect, atol=1e-15)
    # Gauss-Legendre: exact to degree 5 on [-1, 1]
    for n in range(6):
        assert np.sum(R.om_edge * s**n) == pytest.approx(0.0 if n % 2 else 2.0 / (n + 1), abs=1e-14)
