"""Pins of the oracle's 3D form: P2 on tetrahedra (the paper's remark at the end of Sec. 3.3: the
construction carries over to 3D tetrahedral elements, face by face).  Reference tetrahedron
(0,0,0),(1,0,0),(0,1,0),(0,0,1); faces opposite each vertex, 7 points each.

Checks against mathematics: exact monomial moments, an independent Gauss-Jacobi rule from scipy,
finite differences, properties of the 3D Euler flux (homogeneity, the eigenvalues of its normal
Jacobian, rotation invariance, reduction to 2D), the geometry of the tetrahedral mesh (volumes,
closed faces, periodic pairing, the pairing of face points by their coordinates), free-stream
preservation, conservation, symmetry under permutations of the axes, positivity on a blast and
convergence on a smooth plane wave."""
import math

import numpy as np
import pytest
from scipy.special import roots_jacobi

import oracle as O
from paper_1601_08145_amd import inputs as I
from tests import helpers as H

G = 1.4
FACES = I.TET_FACES
VERTS = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)


def tet_rule(n=5):
    """Independent collapsed rule on the reference tetrahedron (weights sum to 1)."""
    x0, w0 = roots_jacobi(n, 0, 0)
    x1, w1 = roots_jacobi(n, 1, 0)
    x2, w2 = roots_jacobi(n, 2, 0)
    pts, wts = [], []
    for i in range(n):
        for j in range(n):
            for k in range(n):
                u, v, w = 0.5 * (1 + x0[i]), 0.5 * (1 + x1[j]), 0.5 * (1 + x2[k])
                pts.append([u * (1 - v) * (1 - w), v * (1 - w), w])
                wts.append(6 / 64 * w0[i] * w1[j] * w2[k])
    return np.array(pts), np.array(wts)


def moment(a, b, c):
    return 6.0 * math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)


def test_tet_basis_and_rules():
    """Basis orthonormal under an independent rule, phi_1 = 1, every phi a quadratic; the interior
    rule exact for every monomial to degree 5 and not 6; the face points on the faces, with the
    7-point rule exact to degree 5 over each face (barycentric moments 2 a! b! c! / (a+b+c+2)!)."""
    R = O.RefElem(O.TET)
    assert (R.dim, R.ML, R.K, R.NI, R.NQE) == (3, 10, 4, 27, 7)
    pts, w = tet_rule()
    B = np.array([[R.phi(l, p) for l in range(10)] for p in pts])
    assert np.abs((B * w[:, None]).T @ B - np.eye(10)).max() < 1e-13
    assert np.allclose(B[:, 0], 1.0, atol=1e-15)
    mono = np.stack([pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c
                     for a in range(3) for b in range(3) for c in range(3) if a + b + c <= 2], 1)
    coef, *_ = np.linalg.lstsq(mono, B, rcond=None)
    assert np.abs(mono @ coef - B).max() < 1e-12
    x, y, z = R.xi_int.T
    assert R.w_int.sum() == pytest.approx(1.0, abs=1e-15) and np.all(R.w_int > 0)
    assert np.all(x > 0) and np.all(y > 0) and np.all(z > 0) and np.all(x + y + z < 1)
    for a in range(6):
        for b in range(6 - a):
            for c in range(6 - a - b):
                assert np.sum(R.w_int * x**a * y**b * z**c) == pytest.approx(moment(a, b, c), abs=1e-15)
    assert abs(np.sum(R.w_int * x**6) - moment(6, 0, 0)) > 1e-9
    assert R.om_edge.sum() == pytest.approx(2.0, abs=1e-15)
    for k, f in enumerate(FACES):
        A, Bv, C = VERTS[list(f)]
        n = np.cross(Bv - A, C - A)
        assert np.dot(n, VERTS[k] - A) < 0  # outward: away from the opposite vertex
        for j in range(7):
            p = R.xi_edge[k, j]
            assert abs(np.dot(p - A, n)) < 1e-15
        # barycentric coordinates of the face points, from a least-squares solve
        T = np.stack([A, Bv, C], 1)
        lam = np.array([np.linalg.lstsq(np.vstack([T, np.ones(3)]), np.append(R.xi_edge[k, j], 1), rcond=None)[0]
                        for j in range(7)])
        assert np.all(lam > 0)
        for a in range(6):
            for b in range(6 - a):
                for c in range(6 - a - b):
                    ex = 2.0 * math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 2)
                    got = 0.5 * np.sum(R.om_edge * lam[:, 0] ** a * lam[:, 1] ** b * lam[:, 2] ** c)
                    assert got == pytest.approx(ex, abs=1e-14)


def test_tet_derivatives_match_differences():
    R = O.RefElem(O.TET)
    rng = np.random.default_rng(2)
    h = 1e-4
    for _ in range(4):
        p = rng.uniform(0.05, 0.25, 3)
        for l in range(10):
            for a in range(3):
                e = np.zeros(3)
                e[a] = h
                d = [0, 0, 0]
                d[a] = 1
                fd = (R.phi(l, p + e) - R.phi(l, p - e)) / (2 * h)
                assert R.phi(l, p, *d) == pytest.approx(fd, abs=1e-7)
                for b in range(3):
                    d2 = list(d)
                    d2[b] += 1
                    db = [0, 0, 0]
                    db[b] = 1
                    fd2 = (R.phi(l, p + e, *db) - R.phi(l, p - e, *db)) / (2 * h)
                    assert R.phi(l, p, *d2) == pytest.approx(fd2, abs=1e-7)


def rand_state3(rng):
    rho = rng.uniform(0.3, 2.0)
    u = rng.uniform(-1.5, 1.5, 3)
    p = rng.uniform(0.2, 3.0)
    return np.concatenate([[rho], rho * u, [p / (G - 1) + 0.5 * rho * u @ u]]), rho, u, p


def test_flux_3d():
    """F(q) = A(q) q; the normal Jacobian sum_d n_d A_d has eigenvalues u.n - c, u.n (three
    times), u.n + c (|n| = 1); rotating the momentum rotates the normal flux; zero z-momentum and
    d < 2 give the 2D flux; Jacobian and Hessian products against differences."""
    rng = np.random.default_rng(0)
    for _ in range(10):
        q, rho, u, p = rand_state3(rng)
        c = math.sqrt(G * p / rho)
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        A = np.zeros((5, 5))
        for d in range(3):
            assert np.allclose(O.flux(q, d), sum(O.flux_jvp(q, np.eye(5)[m], d) * q[m] for m in range(5)), atol=1e-12)
            for m in range(5):
                A[:, m] += n[d] * O.flux_jvp(q, np.eye(5)[m], d)
        ev = np.sort(np.linalg.eigvals(A).real)
        un = u @ n
        assert np.allclose(ev, [un - c, un, un, un, un + c], atol=1e-10)
        # rotation
        Qm, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        rq = q.copy()
        rq[1:4] = Qm @ q[1:4]
        fn = sum(n[d] * O.flux(q, d) for d in range(3))
        rn = Qm @ n
        frn = sum(rn[d] * O.flux(rq, d) for d in range(3))
        assert np.allclose(frn[[0, 4]], fn[[0, 4]], atol=1e-12)
        assert np.allclose(frn[1:4], Qm @ fn[1:4], atol=1e-12)
        # differences
        x, y = rng.normal(size=5) * 0.1, rng.normal(size=5) * 0.1
        hh = 1e-5
        for d in range(3):
            fd = (O.flux(q + hh * x, d) - O.flux(q - hh * x, d)) / (2 * hh)
            assert np.allclose(O.flux_jvp(q, x, d), fd, rtol=1e-7, atol=1e-9)
            fd2 = (O.flux(q + hh * x + hh * y, d) - O.flux(q + hh * x - hh * y, d) - O.flux(q - hh * x + hh * y, d)
                   + O.flux(q - hh * x - hh * y, d)) / (4 * hh * hh)
            assert np.allclose(O.flux_hvp(q, x, y, d), fd2, rtol=1e-4, atol=1e-5)
        # 2D reduction
        q2 = np.array([q[0], q[1], q[2], 0.0, q[4]])
        for d in range(2):
            f3 = O.flux(q2, d)
            f2 = O.flux(q2[[0, 1, 2, 4]], d)
            assert np.allclose(f3[[0, 1, 2, 4]], f2, atol=1e-13) and abs(f3[3]) < 1e-15


def periodic_mesh(n, seed=3, jitter=0.12):
    xyz, tet = I.lattice_tets(n, seed, jitter=jitter, periodic=True)
    tags = I.boundary_tags_tet(xyz, tet, (0, 1, 0, 1, 0, 1), [0] * 6)
    return xyz, tet, O.Mesh.tet(xyz, tet, tags, (1.0, 1.0, 1.0))


def test_tet_mesh_geometry_and_point_pairing():
    """Volumes add up to the box; every tetrahedron's outward face normals (area-weighted) sum to
    zero; each interior face pairs the two tetrahedra that share it, each periodic face its
    translate; and local face point jl of the second element lies where point fmap[jl] of the
    first one does (coordinates computed here from the rule and the vertices, modulo the period)."""
    xyz, tet, M = periodic_mesh(5)
    assert M.N == 6 * 4**3 and M.E == 2 * M.N
    assert M.area.sum() == pytest.approx(1.0, rel=1e-13)
    ei, ki, ej, kj, n = M.edges()
    acc = np.zeros((M.N, 3))
    np.add.at(acc, ei, n)
    np.add.at(acc, ej[ej >= 0], -n[ej >= 0])
    assert np.abs(acc).max() < 1e-15
    assert np.all(ej >= 0)  # fully periodic
    assert np.all(M.nbr[ei, ki] == ej) and np.all(M.nbr[ej, kj] == ei)
    R = O.RefElem(O.TET)
    fmap = M.point_order()
    v = xyz[tet]

    def phys(i, k, j):
        xi = R.xi_edge[k, j]
        return v[i, 0] + xi[0] * (v[i, 1] - v[i, 0]) + xi[1] * (v[i, 2] - v[i, 0]) + xi[2] * (v[i, 3] - v[i, 0])

    checked = 0
    for e in range(M.E):
        i, k, j, kk = ei[e], ki[e], ej[e], kj[e]
        assert np.all(fmap[i, k] == np.arange(7))
        assert sorted(fmap[j, kk]) == list(range(7))
        for jl in range(7):
            d = phys(j, kk, jl) - phys(i, k, fmap[j, kk, jl])
            d -= np.round(d)  # periodic images differ by whole periods
            assert np.abs(d).max() < 1e-12
            checked += 1
    assert checked == 7 * M.E


@pytest.mark.parametrize("periodic", [True, False])
def test_tet_free_stream(periodic):
    """A uniform flow stays uniform to round-off on jittered tetrahedra (periodic, or transparent
    sides)."""
    if periodic:
        _, _, M = periodic_mesh(4)
    else:
        xyz, tet = I.lattice_tets(4, 5)
        M = O.Mesh.tet(xyz, tet)
    Q = np.zeros((M.N, 5, 10))
    Q[:, :, 0] = [1.2, 0.36, -0.24, 0.6, 3.0]
    S = O.Solver(M)
    S.set_state(Q)
    for _ in range(4):
        S.step()
    Q1, _ = S.get_state()
    assert np.abs(Q1 - Q).max() < 1e-13


def test_tet_conservation_with_active_limiters():
    """Rough random states on a periodic mesh: mass, momentum and energy to round-off over five
    steps, while the moment, flux and shock-capturing limiters act; every average stays positive."""
    _, _, M = periodic_mesh(5)
    Q = I.random_modal_state(M.N, 3, 10, seed=9, amp=0.3, rough_frac=0.15, rough_amp=2.5, p_range=(1e-3, 1))
    S = O.Solver(M, alpha0=5.0)
    S.set_state(Q)
    tot0 = np.einsum("i,iv->v", M.area, Q[:, :, 0])
    n_mom = n_flux = n_sc = 0
    for _ in range(5):
        S.step()
        n_mom += np.sum(S.stage(O.STAGE_THETA_MOM) < 1)
        n_flux += np.sum(S.stage(O.STAGE_LAM_E) < 1)
        n_sc += np.sum(S.stage(O.STAGE_THETA_SC) < 1)
    Q1, _ = S.get_state()
    tot1 = np.einsum("i,iv->v", M.area, Q1[:, :, 0])
    assert np.allclose(tot1, tot0, rtol=1e-13, atol=1e-13)
    assert np.all(Q1[:, 0, 0] > 0)
    assert n_mom > 0 and n_sc > 0


def plane_wave(kvec, u0):
    kvec, u0 = np.asarray(kvec, float), np.asarray(u0, float)

    def f(x, t):
        rho = 1 + 0.3 * np.sin(2 * np.pi * (x @ kvec - (u0 @ kvec) * t))
        one = np.ones_like(rho)
        return H.cons(np.stack([rho, u0[0] * one, u0[1] * one, u0[2] * one, one], -1))
    return f


def test_tet_axis_permutation_symmetry():
    """On the unjittered lattice a cyclic permutation of the axes maps the six-tetrahedron split
    onto itself with every tetrahedron's vertex order kept (an even permutation keeps the
    orientation), so a wave along x, along y and along z give the same solution with the axes and
    momenta cycled, to round-off.  (A swap of two axes reverses orientation; the collapsed
    interior rule is not symmetric under the vertex relabelling that then follows.)"""
    xyz, tet = I.lattice_tets(4, 0, jitter=0.0, periodic=True)
    tags = I.boundary_tags_tet(xyz, tet, (0, 1, 0, 1, 0, 1), [0] * 6)
    M = O.Mesh.tet(xyz, tet, tags, (1.0, 1.0, 1.0))
    xc = xyz[tet].mean(1)
    res = []
    for a in range(3):
        e = np.zeros(3)
        e[a] = 1.0
        f = plane_wave(e, 0.5 * e + 0.1)
        S = O.Solver(M)
        S.set_state(M.project(f(M.quad_points(), 0.0)))
        for _ in range(3):
            S.step()
        res.append(S.get_state()[0][:, :, 0])
    key = lambda c: tuple(np.round(c, 9))
    where = {key(c): i for i, c in enumerate(xc)}
    for a in (1, 2):
        idx = np.array([where[key(np.roll(c, a))] for c in xc])  # element of run a that is the image of i
        got = res[a][idx]
        assert np.abs(got[:, [0, 4]] - res[0][:, [0, 4]]).max() < 1e-12
        assert np.abs(got[:, 1:4] - np.roll(res[0][:, 1:4], a, axis=1)).max() < 1e-12


def test_tet_positivity_near_vacuum_blast():
    """Energy 1 in the eight tetrahedra nearest the centre, p = 1e-10 elsewhere (transparent
    sides): every cell average keeps positive density and pressure for 25 steps."""
    xyz, tet = I.lattice_tets(7, 4)
    M = O.Mesh.tet(xyz, tet)
    c = xyz[tet].mean(1)
    Q = np.zeros((M.N, 5, 10))
    Q[:, 0, 0] = 1.0
    Q[:, 4, 0] = 1e-10 / (G - 1)
    near = np.argsort(np.linalg.norm(c - 0.5, axis=1))[:8]
    Q[near, 4, 0] = 1.0 / (8 * M.area[near])
    S = O.Solver(M)
    S.set_state(Q)
    for _ in range(25):
        S.step()
        Q1, _ = S.get_state()
        p = (G - 1) * (Q1[:, 4, 0] - 0.5 * np.sum(Q1[:, 1:4, 0] ** 2, 1) / Q1[:, 0, 0])
        assert np.all(Q1[:, 0, 0] > 0) and np.all(p > 0)
    assert np.sum(S.stage(O.STAGE_THETA_MOM) < 1) > 0


def test_tet_time_derivatives_at_points_converge():
    """q_t = -div F^h and q_tt = sum_d [H_d(d_d q, D) + A_d d_d D] at the interior points of
    tetrahedra against the exact time derivatives of a density wave along (1, 2, -1) with a
    uniform flow: orders about 2 and 1 (first and second derivatives of a cubic-accurate
    projection), from the 4^3- to the 8^3-cube lattice."""
    kv, u0 = np.array([1.0, 2.0, -1.0]), np.array([0.6, -0.3, 0.4])
    f = plane_wave(kv, u0)
    e1, e2 = [], []
    for n in (5, 9):
        _, _, M = periodic_mesh(n)
        xq = M.quad_points()
        S = O.Solver(M, shock=False)
        S.set_state(M.project(f(xq, 0.0)))
        S.step()
        d = S.stage(O.STAGE_QDERIV)
        h = 1e-3
        qt = (f(xq, h) - f(xq, -h)) / (2 * h)
        qtt = (f(xq, h) - 2 * f(xq, 0.0) + f(xq, -h)) / h**2
        e1.append(np.sqrt(np.mean((d[..., 0, :] - qt) ** 2)))
        e2.append(np.sqrt(np.mean((d[..., 1, :] - qtt) ** 2)))
    assert math.log2(e1[0] / e1[1]) > 1.6, e1
    assert math.log2(e2[0] / e2[1]) > 0.7, e2


def test_tet_reflective_box_conserves_mass_and_energy():
    """Reflective walls on all six sides of the box and a smooth state with velocity in every
    direction: no mass or energy crosses a wall (the ghost state reverses the normal momentum),
    so both totals hold to round-off over five steps, while the momentum changes."""
    xyz, tet = I.lattice_tets(5, 6)
    M = O.Mesh.tet(xyz, tet, I.boundary_tags_tet(xyz, tet, (0, 1, 0, 1, 0, 1), [O.BC_REFLECTIVE] * 6))
    xq = M.quad_points()
    x, y, z = xq[..., 0], xq[..., 1], xq[..., 2]
    prim = np.stack([1 + 0.2 * np.sin(2 * x + y), 0.5 + 0.3 * np.cos(3 * y), -0.4 + 0.2 * z, 0.3 + 0.2 * x * y,
                     1 + 0.1 * np.cos(x + 2 * z)], -1)
    Q = M.project(H.cons(prim))
    S = O.Solver(M)
    S.set_state(Q)
    tot0 = np.einsum("i,iv->v", M.area, Q[:, :, 0])
    for _ in range(5):
        S.step()
    Q1, _ = S.get_state()
    tot1 = np.einsum("i,iv->v", M.area, Q1[:, :, 0])
    assert abs(tot1[0] - tot0[0]) < 1e-14 * tot0[0] and abs(tot1[4] - tot0[4]) < 1e-14 * tot0[4]
    assert np.abs(tot1[1:4] - tot0[1:4]).max() > 1e-4


def test_tet_plane_wave_convergence():
    """A density wave along (1, 1, 1) on periodic jittered tetrahedra to t = 0.02: the L2 error of
    rho (independent rule) falls at order > 2.3 from the 4^3- to the 8^3-cube lattice
    (pre-asymptotic, as on triangles at these sizes)."""
    f = plane_wave([1.0, 1.0, 1.0], [0.6, -0.3, 0.4])
    pts, w = tet_rule(4)
    errs = []
    for n in (5, 9):
        _, _, M = periodic_mesh(n)
        S = O.Solver(M)
        S.set_state(M.project(f(M.quad_points(), 0.0)))
        S.advance(0.02)
        qh, x = S.eval_points(pts)
        errs.append(math.sqrt(np.sum((qh[..., 0] - f(x, 0.02)[..., 0]) ** 2 * w[None, :] * M.area[:, None]) / M.area.sum()))
    assert math.log2(errs[0] / errs[1]) > 2.3, errs
