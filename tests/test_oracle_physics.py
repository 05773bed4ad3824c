"""Pins of the oracle's physics (Sec. 1.1, 1.5, 2.2): the Euler flux, its Jacobian and Hessian
products, the time-averaged flux F_T, and the damping-factor solve of Sec. 3.3 Step 5b.

Checks are against mathematics, not against a retyped formula: homogeneity of the Euler flux
(A(q) q = F(q) and H(q)(q, x) = 0), the eigenvalues u.n - c, u.n, u.n + c of the flux Jacobian,
finite differences, the O(dt^3) error of F_T against the exact time average along an exact
smooth solution, rotational invariance, and brute-force maximality of mu."""
import math

import numpy as np
import pytest

import oracle as O

G = 1.4


def rand_state(rng, dim):
    rho = rng.uniform(0.3, 2.0)
    u = rng.uniform(-1.5, 1.5, dim)
    p = rng.uniform(0.2, 3.0)
    E = p / (G - 1) + 0.5 * rho * np.dot(u, u)
    return np.concatenate([[rho], rho * u, [E]]), rho, u, p


@pytest.mark.parametrize("dim", [1, 2])
def test_flux_homogeneity_and_mass_flux(dim):
    rng = np.random.default_rng(0)
    for _ in range(20):
        q, rho, u, p = rand_state(rng, dim)
        for d in range(dim):
            F = O.flux(q, d)
            assert F[0] == pytest.approx(q[1 + d], rel=1e-15)
            # Euler's theorem for the degree-1 homogeneous flux: A(q) q = F(q)
            assert np.allclose(O.flux_jvp(q, q, d), F, rtol=1e-13, atol=1e-13)
            # A is homogeneous of degree 0, so H(q)(q, x) = 0
            x = rng.normal(size=len(q))
            assert np.allclose(O.flux_hvp(q, q, x, d), 0.0, atol=1e-12)
            # energy flux u (E + p)
            assert F[-1] == pytest.approx(u[d] * (q[-1] + p), rel=1e-13)


def test_flux_1d_equals_2d_without_transverse_velocity():
    rng = np.random.default_rng(1)
    for _ in range(10):
        q1, rho, u, p = rand_state(rng, 1)
        q2 = np.array([q1[0], q1[1], 0.0, q1[2]])
        F1 = O.flux(q1, 0)
        F2 = O.flux(q2, 0)
        assert np.allclose(F2[[0, 1, 3]], F1, rtol=1e-14)
        assert F2[2] == 0.0


def test_flux_rotational_invariance():
    rng = np.random.default_rng(2)
    for _ in range(10):
        q, rho, u, p = rand_state(rng, 2)
        a = rng.uniform(0, 2 * np.pi)
        n = np.array([np.cos(a), np.sin(a)])
        Fn = n[0] * O.flux(q, 0) + n[1] * O.flux(q, 1)
        Rm = np.array([[n[0], n[1]], [-n[1], n[0]]])  # rotates n onto the x axis
        qr = q.copy()
        qr[1:3] = Rm @ q[1:3]
        Fx = O.flux(qr, 0)
        back = Fx.copy()
        back[1:3] = Rm.T @ Fx[1:3]
        assert np.allclose(Fn, back, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("dim", [1, 2])
def test_jacobian_eigenvalues(dim):
    rng = np.random.default_rng(3)
    for _ in range(10):
        q, rho, u, p = rand_state(rng, dim)
        c = math.sqrt(G * p / rho)
        a = rng.uniform(0, 2 * np.pi)
        n = np.array([np.cos(a), np.sin(a)])[:dim] if dim == 2 else np.array([1.0])
        V = len(q)
        A = np.zeros((V, V))
        for j in range(V):
            e = np.zeros(V)
            e[j] = 1.0
            A[:, j] = sum(n[d] * O.flux_jvp(q, e, d) for d in range(dim))
        ev = np.sort(np.linalg.eigvals(A).real)
        un = float(np.dot(u, n))
        expect = np.sort([un - c, un + c] + [un] * (V - 2))
        assert np.allclose(ev, expect, atol=1e-10)


@pytest.mark.parametrize("dim", [1, 2])
def test_jvp_hvp_against_finite_differences(dim):
    rng = np.random.default_rng(4)
    h = 1e-5
    for _ in range(10):
        q, *_ = rand_state(rng, dim)
        x = rng.normal(size=len(q)) * 0.1
        y = rng.normal(size=len(q)) * 0.1
        for d in range(dim):
            fd = (O.flux(q + h * x, d) - O.flux(q - h * x, d)) / (2 * h)
            assert np.allclose(O.flux_jvp(q, x, d), fd, rtol=1e-7, atol=1e-9)
            fd2 = (O.flux(q + h * x + h * y, d) - O.flux(q + h * x - h * y, d) - O.flux(q - h * x + h * y, d)
                   + O.flux(q - h * x - h * y, d)) / (4 * h * h)
            assert np.allclose(O.flux_hvp(q, x, y, d), fd2, rtol=1e-4, atol=1e-5)
            assert np.allclose(O.flux_hvp(q, x, y, d), O.flux_hvp(q, y, x, d), rtol=1e-13, atol=1e-14)


def vortex_prim(x, y, t, eps=5.0, uinf=(1.0, 0.5)):
    """Exact isentropic vortex (Shu's), advected with uinf."""
    xr, yr = x - uinf[0] * t, y - uinf[1] * t
    r2 = xr * xr + yr * yr
    f = np.exp(0.5 * (1 - r2))
    T = 1 - (G - 1) * eps**2 / (8 * G * np.pi**2) * f * f
    rho = T ** (1 / (G - 1))
    return rho, uinf[0] - eps / (2 * np.pi) * f * yr, uinf[1] + eps / (2 * np.pi) * f * xr, rho * T


def vortex_cons(x, y, t):
    r, u, v, p = vortex_prim(x, y, t)
    return np.array([r, r * u, r * v, p / (G - 1) + 0.5 * r * (u * u + v * v)])


def test_ft_is_third_order_time_average():
    """|| (1/dt) int_0^dt F(q(t)) dt - F_T || = O(dt^3) along an exact solution (Eq. (1D_system.TI-F)),
    with q_t, q_tt of that solution taken by differences in time."""
    x, y = 0.7, -0.4
    errs = []
    for dt in [0.08, 0.04, 0.02]:
        hh = 1e-3
        q0 = vortex_cons(x, y, 0.0)
        qt = (vortex_cons(x, y, hh) - vortex_cons(x, y, -hh)) / (2 * hh)
        qtt = (vortex_cons(x, y, hh) - 2 * q0 + vortex_cons(x, y, -hh)) / hh**2
        FT = O.ft(q0, qt, qtt, dt)
        tg, wg = np.polynomial.legendre.leggauss(12)
        ts = 0.5 * dt * (tg + 1)
        avg = sum(0.5 * w * np.array([O.flux(vortex_cons(x, y, t), d) for d in range(2)]) for t, w in zip(ts, wg))
        errs.append(np.abs(avg - FT).max())
    r1 = math.log2(errs[0] / errs[1])
    r2 = math.log2(errs[1] / errs[2])
    assert r1 > 2.7 and r2 > 2.7, errs


def test_mu_solve_is_the_largest_positive_fraction():
    rng = np.random.default_rng(5)
    n_lim = 0
    for _ in range(300):
        dim = 2
        qL, rho, u, p = rand_state(rng, dim)
        qa = qL + rng.normal(size=4) * np.array([0.8, 1.5, 1.5, 2.5]) * rng.uniform(0.1, 2.0)
        pL = (G - 1) * (qL[3] - 0.5 * (qL[1] ** 2 + qL[2] ** 2) / qL[0])
        eps_p = min(1e-12, pL)
        mu = O.mu_solve(qL, qa, eps_p)
        assert 0.0 <= mu <= 1.0

        def ok(m):
            q = qL + m * (qa - qL)
            return q[0] > 0 and (G - 1) * (q[3] - 0.5 * (q[1] ** 2 + q[2] ** 2) / q[0]) >= eps_p

        assert ok(mu)
        if mu < 1.0:
            n_lim += 1
            # brute force: bisection on the first crossing
            lo, hi = 0.0, 1.0
            grid = np.linspace(0, 1, 2001)
            bad = [g for g in grid if not ok(g)]
            hi = bad[0]
            lo = grid[list(grid).index(hi) - 1]
            for _ in range(60):
                mid = 0.5 * (lo + hi)
                lo, hi = (mid, hi) if ok(mid) else (lo, mid)
            assert mu == pytest.approx(lo, abs=1e-12)
    assert n_lim > 20


def test_mu_solve_target_at_the_lxf_pressure():
    """Near vacuum the target is the LxF corner's own pressure (p(q^LxF) <= eps0): the quadratic's
    constant term vanishes, and where the pressure falls along the segment no fraction above 0
    keeps it (every sampled mu > 0 fails), so mu = 0; where it rises, mu is positive and keeps it."""
    rng = np.random.default_rng(6)
    n_fall = n_rise = 0
    for _ in range(200):
        rho = rng.uniform(1e-4, 1e-2)
        u = rng.normal(size=2)
        pL = rng.uniform(1e-14, 1e-12)
        qL = np.array([rho, rho * u[0], rho * u[1], pL / (G - 1) + 0.5 * rho * (u @ u)])
        qa = qL + rng.normal(size=4) * np.array([0.3 * rho, rho, rho, 1e-12])
        eps_p = min(1e-12, (G - 1) * (qL[3] - 0.5 * (qL[1] ** 2 + qL[2] ** 2) / qL[0]))
        mu = O.mu_solve(qL, qa, eps_p)

        def p_at(m):
            q = qL + m * (qa - qL)
            return (G - 1) * (q[3] - 0.5 * (q[1] ** 2 + q[2] ** 2) / q[0]) if q[0] > 0 else -np.inf

        small = [p_at(m) for m in (1e-9, 1e-6, 1e-3)]
        if all(p < eps_p for p in small):
            assert mu == 0.0
            n_fall += 1
        elif mu > 0.0:
            assert p_at(mu) >= eps_p
            n_rise += 1
    assert n_fall > 20 and n_rise > 20
