"""Pins of the oracle's degree-3 (fourth-order) form: the scheme carried one order further, as the
paper states it extends to any order (abstract, Sec. 2.2 and 5): P3 bases on the line and the
triangle, rules exact to degree 7, the third derivative of the flux, the time-averaged flux F_T to
fourth order (Eq. (1D_system.TI-F) with the dt^3 term), the third time derivative at the points,
and fourth-order convergence of the whole step on smooth solutions.

Checks are against mathematics: closed forms of the Gauss-Legendre rule and the Legendre
polynomials, exact monomial integrals, an independent numpy rule, finite differences of the plain
flux, the exact time average along a cubic state path, the exact time derivatives of an advected
vortex, and exact (or finely resolved) smooth solutions."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1601_08145_amd import inputs as I
from tests import helpers as H

G = 1.4


def order(e):
    return [math.log2(e[i] / e[i + 1]) for i in range(len(e) - 1)]


def test_p3_line_rules_and_basis_closed_forms():
    """Four-point Gauss-Legendre nodes +-sqrt(3/7 -+ 2/7 sqrt(6/5)) with weights (18 +- sqrt 30)/36
    (normalised by the length 2), and the orthonormal Legendre basis sqrt(2l+1) P_l up to P_3."""
    R = O.RefElem(O.LINE, 3)
    assert R.ML == 4 and R.NI == 4
    a, b = math.sqrt(3 / 7 - 2 / 7 * math.sqrt(6 / 5)), math.sqrt(3 / 7 + 2 / 7 * math.sqrt(6 / 5))
    order_ = np.argsort(R.xi_int[:, 0])
    assert np.allclose(R.xi_int[order_, 0], [-b, -a, a, b], atol=1e-15)
    wa, wb = (18 + math.sqrt(30)) / 72, (18 - math.sqrt(30)) / 72
    assert np.allclose(R.w_int[order_], [wb, wa, wa, wb], atol=1e-15)
    for n in range(8):
        assert np.sum(R.w_int * R.xi_int[:, 0] ** n) == pytest.approx(0.0 if n % 2 else 1.0 / (n + 1), abs=1e-15)
    for x in [-1.0, -0.6, 0.1, 0.77, 1.0]:
        P = [1.0, x, 0.5 * (3 * x * x - 1), 0.5 * (5 * x ** 3 - 3 * x)]
        for l in range(4):
            assert R.phi(l, [x]) == pytest.approx(math.sqrt(2 * l + 1) * P[l], abs=1e-14)
            # derivatives of the closed forms
            dP = [0.0, 1.0, 3 * x, 0.5 * (15 * x * x - 3)][l]
            d2P = [0.0, 0.0, 3.0, 15 * x][l]
            d3P = [0.0, 0.0, 0.0, 15.0][l]
            s = math.sqrt(2 * l + 1)
            assert R.phi(l, [x], 1) == pytest.approx(s * dP, abs=1e-13)
            assert R.phi(l, [x], 2) == pytest.approx(s * d2P, abs=1e-13)
            assert R.phi(l, [x], 3) == pytest.approx(s * d3P, abs=1e-13)


def test_p3_triangle_rules():
    """The interior rule integrates every monomial of total degree <= 7 exactly (2 a! b!/(a+b+2)!
    normalised by the area 1/2) and not degree 8; the edge rules put four Gauss points on each edge,
    exact to degree 7 along it."""
    R = O.RefElem(O.TRI, 3)
    assert R.ML == 10 and R.NQE == 4
    assert R.w_int.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.all(R.w_int > 0)
    x, y = R.xi_int[:, 0], R.xi_int[:, 1]
    assert np.all(x > 0) and np.all(y > 0) and np.all(x + y < 1)
    exact = lambda a, b: 2.0 * math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
    for a in range(8):
        for b in range(8 - a):
            assert np.sum(R.w_int * x ** a * y ** b) == pytest.approx(exact(a, b), abs=1e-15), (a, b)
    assert abs(np.sum(R.w_int * x ** 8) - exact(8, 0)) > 1e-9
    verts = [(0, 0), (1, 0), (0, 1)]
    assert R.om_edge.sum() == pytest.approx(2.0, abs=1e-15)
    gx, _ = np.polynomial.legendre.leggauss(4)
    for k in range(3):
        A, B = np.array(verts[k]), np.array(verts[(k + 1) % 3])
        for j in range(4):
            s = 2 * np.dot(R.xi_edge[k, j] - A, B - A) / np.dot(B - A, B - A) - 1
            assert np.allclose(R.xi_edge[k, j], A + 0.5 * (1 + s) * (B - A), atol=1e-15)
        s_k = np.array([2 * np.dot(R.xi_edge[k, j] - A, B - A) / np.dot(B - A, B - A) - 1 for j in range(4)])
        assert np.allclose(np.sort(s_k), gx, atol=1e-15)
    for n in range(8):
        s_all = np.array([2 * np.dot(R.xi_edge[0, j] - np.array(verts[0]), [1, 0]) - 1 for j in range(4)])
        assert np.sum(R.om_edge * s_all ** n) == pytest.approx(0.0 if n % 2 else 2.0 / (n + 1), abs=1e-14)


@pytest.mark.parametrize("kind", [O.LINE, O.TRI])
def test_p3_basis_orthonormal_and_spans_the_cubics(kind):
    """Orthonormal under (1/|T0|) int (an independent collapsed Gauss rule), phi_1 = 1, every basis
    function a polynomial of degree <= 3 (a least-squares fit to the cubic monomials leaves nothing),
    and the projection of every cubic monomial onto the basis reproduces it exactly."""
    R = O.RefElem(kind, 3)
    pts, w = H.error_rule(kind, 10)
    B = np.array([[R.phi(l, p) for l in range(R.ML)] for p in pts])
    assert np.allclose((B * w[:, None]).T @ B, np.eye(R.ML), atol=1e-13)
    assert np.allclose(B[:, 0], 1.0, atol=1e-15)
    if kind == O.LINE:
        mono = np.stack([pts[:, 0] ** a for a in range(4)], 1)
    else:
        mono = np.stack([pts[:, 0] ** a * pts[:, 1] ** b for a in range(4) for b in range(4 - a)], 1)
    assert mono.shape[1] == R.ML
    coef, *_ = np.linalg.lstsq(mono, B, rcond=None)
    assert np.abs(mono @ coef - B).max() < 1e-12
    proj = B @ ((B * w[:, None]).T @ mono)
    assert np.abs(proj - mono).max() < 1e-12


def test_p3_triangle_derivatives_match_differences():
    R = O.RefElem(O.TRI, 3)
    rng = np.random.default_rng(3)
    h = 1e-4
    for _ in range(4):
        p = rng.uniform(0.05, 0.4, 2)
        for l in range(R.ML):
            for a, da in ((0, (1, 0)), (1, (0, 1))):
                e = np.zeros(2)
                e[a] = h
                fd = (R.phi(l, p + e) - R.phi(l, p - e)) / (2 * h)
                assert R.phi(l, p, *da) == pytest.approx(fd, abs=1e-5)  # h^2/6 phi''' of a cubic
                # mixed and third derivatives from differences of the derivative tables
                for b, db in ((0, (1, 0)), (1, (0, 1))):
                    d2 = (da[0] + db[0], da[1] + db[1])
                    fd2 = (R.phi(l, p + e, *db) - R.phi(l, p - e, *db)) / (2 * h)
                    assert R.phi(l, p, *d2) == pytest.approx(fd2, abs=1e-6)
                    for c, dc in ((0, (1, 0)), (1, (0, 1))):
                        d3 = (d2[0] + dc[0], d2[1] + dc[1])
                        fd3 = (R.phi(l, p + e, *(dc[0] + db[0], dc[1] + db[1]))
                               - R.phi(l, p - e, *(dc[0] + db[0], dc[1] + db[1]))) / (2 * h)
                        assert R.phi(l, p, *d3) == pytest.approx(fd3, abs=1e-6)
            # fourth derivatives of a cubic vanish
            assert R.phi(l, p, 4, 0) == 0.0 and R.phi(l, p, 2, 2) == 0.0 and R.phi(l, p, 1, 3) == 0.0


def rand_state(rng, dim):
    rho = rng.uniform(0.3, 2.0)
    u = rng.uniform(-1.5, 1.5, dim)
    p = rng.uniform(0.2, 3.0)
    return np.concatenate([[rho], rho * u, [p / (G - 1) + 0.5 * rho * np.dot(u, u)]])


@pytest.mark.parametrize("dim", [1, 2])
def test_flux_third_derivative_against_differences(dim):
    """F'''(q)[x, y, z]: the third derivative of t -> F(q + t x) by a seven-point difference of the
    plain flux (x = y = z), the mixed third derivative by differences of F over the cube of
    (+-h x, +-h y, +-h z) offsets, symmetry in its three arguments, and zero when an argument is q
    itself twice over (F is homogeneous of degree 1, so F'' (q, .) = 0 and F''' (q, y, z) = -F''(y, z))."""
    rng = np.random.default_rng(7)
    for _ in range(8):
        q = rand_state(rng, dim)
        x, y, z = (rng.normal(size=len(q)) * 0.1 for _ in range(3))
        for d in range(dim):
            h = 2e-2
            f = lambda t: O.flux(q + t * x, d)
            fd3 = (-f(3 * h) + 8 * f(2 * h) - 13 * f(h) + 13 * f(-h) - 8 * f(-2 * h) + f(-3 * h)) / (8 * h ** 3)
            assert np.allclose(O.flux_3vp(q, x, x, x, d), fd3, rtol=1e-4, atol=1e-6)
            h = 1e-3
            mixed = sum(sx * sy * sz * O.flux(q + h * (sx * x + sy * y + sz * z), d)
                        for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)) / (8 * h ** 3)
            got = O.flux_3vp(q, x, y, z, d)
            assert np.allclose(got, mixed, rtol=1e-3, atol=1e-5)
            for perm in [(y, x, z), (z, y, x), (x, z, y)]:
                assert np.allclose(O.flux_3vp(q, *perm, d), got, rtol=1e-12, atol=1e-14)
            assert np.allclose(O.flux_3vp(q, q, y, z, d), -O.flux_hvp(q, y, z, d), rtol=1e-12, atol=1e-12)


def test_ft4_is_fourth_order_time_average():
    """|| (1/dt) int_0^dt F(q(t)) dt - F_T || = O(dt^4) along a cubic state path
    q(t) = q + t q_t + t^2/2 q_tt + t^3/6 q_ttt, whose time derivatives at 0 are those given
    (the time average by 12-point Gauss); without the dt^3 term the error falls only at order 3."""
    rng = np.random.default_rng(11)
    for dim in (1, 2):
        q = rand_state(rng, dim)
        qt, qtt, qttt = (rng.normal(size=len(q)) * s for s in (0.5, 0.8, 1.2))
        errs, errs3 = [], []
        for dt in [0.08, 0.04, 0.02, 0.01]:
            tg, wg = np.polynomial.legendre.leggauss(12)
            ts = 0.5 * dt * (tg + 1)
            path = lambda t: q + t * qt + t * t / 2 * qtt + t ** 3 / 6 * qttt
            avg = sum(0.5 * w * np.array([O.flux(path(t), d) for d in range(dim)]) for t, w in zip(ts, wg))
            errs.append(np.abs(avg - O.ft4(q, qt, qtt, qttt, dt)).max())
            errs3.append(np.abs(avg - O.ft(q, qt, qtt, dt)).max())
        assert min(order(errs)) > 3.8, errs
        assert max(order(errs3)) < 3.2, errs3
        # the degree-2 F_T is the same expansion without the dt^3 term
        assert np.allclose(O.ft4(q, qt, qtt, np.zeros_like(q), 0.0), O.ft(q, qt, qtt, 0.0), rtol=1e-14, atol=1e-14)


def test_p3_time_derivatives_at_points_converge():
    """q_t, q_tt and q_ttt at the interior points of P3 triangles (the chain rule of Sec. 2.2 carried
    one derivative further), against the exact time derivatives of an advected vortex: orders 3, 2
    and 1 (first, second and third derivatives of a fourth-order projection)."""
    U = (1.0, 0.5)

    def qex(x, y, t):
        return H.cons(H.vortex_prim(x, y, t, uinf=U))

    e = [[], [], []]
    for n in [12, 24, 48]:
        xy, tri = I.lattice_delaunay(n + 1, 3, box=(-5, 5, -5, 5))
        M = O.Mesh.tri(xy, tri, degree=3)
        xq = M.quad_points()
        X, Y = xq[..., 0], xq[..., 1]
        S = O.Solver(M, shock=False)
        S.set_state(M.project(qex(X, Y, 0.0)))
        S.step()
        d = S.stage(O.STAGE_QDERIV)
        h = 1e-2
        f = [qex(X, Y, k * h) for k in (-2, -1, 0, 1, 2)]
        ex = [(f[0] - 8 * f[1] + 8 * f[3] - f[4]) / (12 * h),
              (-f[0] + 16 * f[1] - 30 * f[2] + 16 * f[3] - f[4]) / (12 * h * h),
              (-f[0] + 2 * f[1] - 2 * f[3] + f[4]) / (2 * h ** 3)]
        inner = (np.abs(X) < 3) & (np.abs(Y) < 3)
        for k in range(3):
            e[k].append(np.sqrt(np.mean((d[..., k, :] - ex[k])[inner] ** 2)))
    assert min(order(e[0])) > 2.6, e[0]
    assert min(order(e[1])) > 1.7, e[1]
    assert min(order(e[2])) > 0.8, e[2]
    # at degree 2 the third slot stays zero
    xy, tri = I.lattice_delaunay(7, 3, box=(-5, 5, -5, 5))
    M = O.Mesh.tri(xy, tri)
    S = O.Solver(M, shock=False)
    S.set_state(M.project(qex(*np.moveaxis(M.quad_points(), -1, 0), 0.0)))
    S.step()
    assert np.all(S.stage(O.STAGE_QDERIV)[..., 2, :] == 0.0)


def fine_eval(Qf, R, x):
    """q^h of a uniform periodic 1D P3 solution on [0, 1) at the points x."""
    n = Qf.shape[0]
    idx = np.minimum((x * n).astype(int), n - 1)
    xi = 2 * (x * n - idx) - 1
    B = np.array([[R.phi(l, [s]) for l in range(R.ML)] for s in xi])
    return np.einsum("pvl,pl->pv", Qf[idx], B)


def test_p3_1d_fourth_order():
    """Whole P3 step at CFL 0.05 (P3 needs a smaller Courant number than the paper's 0.08 for P2: at
    0.1 the smooth runs below go unstable on the finer meshes), L2 error of rho at T = 0.1:
    - an advected density wave (exact solution): order 4;
    - an isentropic simple wave of amplitude 0.2 before it steepens into a shock (all of F', F'' and
      F''' act), against a 320-cell P3 run: order > 3.6 on 10 -> 20 -> 40 cells."""
    R = O.RefElem(O.LINE, 3)
    T = 0.1

    def wave(x, t=0.0):
        rho = 1 + 0.5 * np.sin(2 * np.pi * (x[..., 0] - t))
        one = np.ones_like(rho)
        return I.prim_to_cons(np.stack([rho, one, one], -1), G)

    errs = []
    for n in [10, 20, 40]:
        M = O.Mesh.line(n, 0, 1, O.BC_PERIODIC, O.BC_PERIODIC, degree=3)
        S = O.Solver(M, cfl=0.05)
        S.set_state(M.project(wave(M.quad_points())))
        S.advance(T)
        errs.append(H.l2_error(S, R, lambda x: wave(x, T)))
    assert min(order(errs)) > 3.85, errs

    def simple(x):
        # Riemann invariant u - 2c/(gamma-1) constant, p = rho^gamma: a right-going simple wave
        rho = 1 + 0.2 * np.sin(2 * np.pi * x[..., 0])
        c = np.sqrt(G * rho ** (G - 1))
        u = 2 / (G - 1) * (c - math.sqrt(G))
        return I.prim_to_cons(np.stack([rho, u, rho ** G], -1), G)

    def run(n):
        M = O.Mesh.line(n, 0, 1, O.BC_PERIODIC, O.BC_PERIODIC, degree=3)
        S = O.Solver(M, cfl=0.05)
        S.set_state(M.project(simple(M.quad_points())))
        S.advance(T)
        return S

    Qf = run(320).get_state()[0]
    errs = []
    for n in [10, 20, 40]:
        S = run(n)
        pts, w = H.error_rule(O.LINE, 8)
        qh, x = S.eval_points(pts)
        ref = fine_eval(Qf, R, x[..., 0].ravel()).reshape(qh.shape)
        errs.append(math.sqrt(np.sum((qh[..., 0] - ref[..., 0]) ** 2 * w[None, :] * S.mesh.area[:, None]) / S.mesh.area.sum()))
    assert min(order(errs)) > 3.6, errs


def test_p3_triangle_vortex_fourth_order():
    """Whole P3 step on periodic jittered triangles (Shu's vortex, CFL 0.05, T = 0.1): L2 error of rho
    falls at order > 3.5 from the 9^2 to the 17^2 lattice (3.9 measured at T = 0.2)."""
    R = O.RefElem(O.TRI, 3)
    T = 0.1
    ex = lambda x, t: H.cons(H.vortex_prim(x[..., 0], x[..., 1], t, period=(10.0, 10.0)))
    errs = []
    for n in [9, 17]:
        xy, tri = I.lattice_delaunay(n, 4, box=(-5, 5, -5, 5), periodic=True)
        tags = I.boundary_tags(xy, tri, (-5, 5, -5, 5), [O.BC_PERIODIC] * 4)
        M = O.Mesh.tri(xy, tri, tags, (10.0, 10.0), degree=3)
        S = O.Solver(M, cfl=0.05)
        S.set_state(M.project(ex(M.quad_points(), 0.0)))
        S.advance(T)
        errs.append(H.l2_error(S, R, lambda x: ex(x, T)))
    assert order(errs)[0] > 3.5, errs


def test_p3_conservation_and_positivity_on_a_blast():
    """The limiters at degree 3: a 1D Sedov-like blast (energy in one cell, near-vacuum pressure
    around) keeps every cell average positive and mass and energy to round-off."""
    n = 64
    M = O.Mesh.line(n, -1, 1, O.BC_PERIODIC, O.BC_PERIODIC, degree=3)
    S = O.Solver(M, cfl=0.05)
    Q = np.zeros((n, 3, 4))
    Q[:, 0, 0] = 1.0
    Q[:, 2, 0] = 1e-12 / (G - 1)
    Q[n // 2, 2, 0] = 3.2e6 * (2.0 / n) ** 0 / (G - 1)
    S.set_state(Q)
    m0, e0 = Q[:, 0, 0].sum(), Q[:, 2, 0].sum()
    k = S.advance(1e-4, max_steps=400)
    Q1, t = S.get_state()
    assert k > 20
    assert np.all(Q1[:, 0, 0] > 0)
    p = (G - 1) * (Q1[:, 2, 0] - 0.5 * Q1[:, 1, 0] ** 2 / Q1[:, 0, 0])
    assert np.all(p > 0)
    assert Q1[:, 0, 0].sum() == pytest.approx(m0, rel=1e-13)
    assert Q1[:, 2, 0].sum() == pytest.approx(e0, rel=1e-12)


def test_p3_time_derivatives_exact_on_cubic_flux_states():
    """When the flux of q^h is itself a cubic (density constant, momentum linear, energy quadratic:
    then m m^T / rho, p and (E + p) m / rho are polynomials of degree <= 3), the P3 projection F^h is
    exact and the chain rule of Sec. 2.2 gives the exact time derivatives of the Euler solution from
    those data (Cauchy-Kovalevskaya): q_t = -div F, q_tt = -div (A q_t), q_ttt = -div (H(q_t, q_t) +
    A q_tt).  Computed here independently by nested central differences in space (nine points, exact
    for the polynomials of degree <= 8 that these fields are) of the plain flux and its derivative
    products at the physical points, against the oracle's values at every interior point of a small
    triangle mesh."""
    rng = np.random.default_rng(5)
    a = rng.uniform(-0.5, 0.5, (2, 3))          # momentum: a[c, 0] + a[c, 1] x + a[c, 2] y
    e = rng.uniform(-0.3, 0.3, 6)                # energy: 3 + quadratic
    rho = 1.3

    def q_at(x, y):
        m = a[:, 0] + a[:, 1] * x + a[:, 2] * y
        E = 3.0 + e[0] * x + e[1] * y + e[2] * x * x + e[3] * x * y + e[4] * y * y + e[5]
        return np.array([rho, m[0], m[1], E])

    h = 0.05
    c9 = np.array([1 / 280, -4 / 105, 1 / 5, -4 / 5, 0.0, 4 / 5, -1 / 5, 4 / 105, -1 / 280])
    offs = np.arange(-4, 5)

    def div(field, x, y):
        """- div of a field (x, y) -> (2, V) flux, by nine-point central differences."""
        gx = sum(c * field(x + k * h, y)[0] for c, k in zip(c9, offs) if c != 0.0) / h
        gy = sum(c * field(x, y + k * h)[1] for c, k in zip(c9, offs) if c != 0.0) / h
        return -(gx + gy)

    F = lambda x, y: np.array([O.flux(q_at(x, y), d) for d in range(2)])
    qt = lambda x, y: div(F, x, y)
    Ft = lambda x, y: np.array([O.flux_jvp(q_at(x, y), qt(x, y), d) for d in range(2)])
    qtt = lambda x, y: div(Ft, x, y)

    def Ftt(x, y):
        q, t1, t2 = q_at(x, y), qt(x, y), qtt(x, y)
        return np.array([O.flux_hvp(q, t1, t1, d) + O.flux_jvp(q, t2, d) for d in range(2)])

    qttt = lambda x, y: div(Ftt, x, y)

    xy, tri = I.lattice_delaunay(4, 2, box=(0, 1, 0, 1))
    M = O.Mesh.tri(xy, tri, degree=3)
    xq = M.quad_points()
    Q = M.project(np.array([[q_at(*p) for p in row] for row in xq]))
    S = O.Solver(M, shock=False)
    S.set_state(Q)
    S.step()
    d = S.stage(O.STAGE_QDERIV)
    for i in range(0, M.N, 5):
        for m in range(0, M.NI, 5):
            x, y = xq[i, m]
            for k, fn in enumerate((qt, qtt, qttt)):
                ex = fn(x, y)
                assert np.allclose(d[i, m, k], ex, rtol=1e-8, atol=1e-8 * max(1.0, np.abs(ex).max())), (i, m, k)
