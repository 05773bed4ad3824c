"""Whole-step pins of the oracle: design-order (third-order) convergence on exact smooth solutions
(Sec. 4.3.1, Table (convergence) reports orders near 3), conservation to round-off on periodic
meshes, positivity of cell averages and of the limited point values on near-vacuum problems
(Sec. 3, Sec. 4.2), and convergence to the exact solution of 1D Riemann problems."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1601_08145_amd import inputs as I
from tests import helpers as H
from tests.exact_riemann import ExactRiemann


def test_sod_star_state_golden():
    vals = np.loadtxt("tests/golden/sod_star_state.txt")
    ex = ExactRiemann((1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    rl = ex.sample(ex.us - 1e-9)[0]
    rr = ex.sample(ex.us + 1e-9)[0]
    assert np.allclose([ex.ps, ex.us, rl, rr], vals, atol=6e-6)


def order(errs):
    return [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


def test_convergence_1d_smooth():
    R = O.RefElem(O.LINE)

    def ic(x, t=0.0):
        rho = 1 + 0.5 * np.sin(2 * np.pi * (x[..., 0] - t))
        one = np.ones_like(rho)
        return I.prim_to_cons(np.stack([rho, one, one], -1), 1.4)

    errs = []
    for n in [10, 20, 40, 80]:
        M = O.Mesh.line(n, 0, 1, O.BC_PERIODIC, O.BC_PERIODIC)
        S = O.Solver(M, cfl=0.1)
        S.set_state(M.project(ic(M.quad_points())))
        S.advance(0.1)
        errs.append(H.l2_error(S, R, lambda x: ic(x, 0.1)))
    assert min(order(errs)[1:]) > 2.8, errs


def test_convergence_2d_vortex_cartesian():
    R = O.RefElem(O.QUAD)
    period = (10.0, 10.0)

    def ex(x, t):
        return H.cons(H.vortex_prim(x[..., 0], x[..., 1], t, period=period))

    errs = []
    for n in [8, 16, 32]:
        M = O.Mesh.cart(n, n, -5, 5, -5, 5, [O.BC_PERIODIC] * 4)
        S = O.Solver(M)
        S.set_state(M.project(ex(M.quad_points(), 0.0)))
        S.advance(0.5)
        errs.append(H.l2_error(S, R, lambda x: ex(x, 0.5)))
    # pre-asymptotic at these sizes (orders ~2.1, 2.4 here; ~2.4 again at 64^2): the paper's own
    # table reaches 3 only past a few thousand cells
    assert order(errs)[-1] > 2.2, errs


def test_time_derivatives_at_points_converge():
    """q_t = -div F^h and q_tt = sum_d [H_d(d_d q, D) + A_d d_d D] (Sec. 2.2-2.3) at the interior
    points, against the exact time derivatives of an advected vortex: q_t converges at order 2
    (first derivatives of a cubic-accurate projection) and q_tt at order 1 (second derivatives)."""
    U = (1.0, 0.5)

    def qex(x, y, t):
        return H.cons(H.vortex_prim(x, y, t, uinf=U))

    for kind in ["cart", "tri"]:
        e1, e2 = [], []
        for n in [16, 32, 64]:
            if kind == "cart":
                M = O.Mesh.cart(n, n, -5, 5, -5, 5, [O.BC_TRANSPARENT] * 4)
            else:
                xy, tri = I.lattice_delaunay(n + 1, 3, box=(-5, 5, -5, 5))
                M = O.Mesh.tri(xy, tri)
            xq = M.quad_points()
            X, Y = xq[..., 0], xq[..., 1]
            S = O.Solver(M, shock=False)
            S.set_state(M.project(qex(X, Y, 0.0)))
            S.step()
            d = S.stage(O.STAGE_QDERIV)
            h = 1e-3
            qt = (qex(X, Y, h) - qex(X, Y, -h)) / (2 * h)
            qtt = (qex(X, Y, h) - 2 * qex(X, Y, 0) + qex(X, Y, -h)) / h**2
            inner = (np.abs(X) < 3) & (np.abs(Y) < 3)
            e1.append(np.sqrt(np.mean((d[..., 0, :] - qt)[inner] ** 2)))
            e2.append(np.sqrt(np.mean((d[..., 1, :] - qtt)[inner] ** 2)))
        assert min(order(e1)) > 1.6, (kind, e1)
        assert min(order(e2)) > 0.75 and order(e2)[-1] > 0.9, (kind, e2)


def test_convergence_2d_vortex_triangles():
    R = O.RefElem(O.TRI)
    period = (10.0, 10.0)

    def ex(x, t):
        return H.cons(H.vortex_prim(x[..., 0], x[..., 1], t, period=period))

    errs = []
    for n in [9, 17, 33]:
        xy, tri = I.lattice_delaunay(n, 4, box=(-5, 5, -5, 5), periodic=True)
        tags = I.boundary_tags(xy, tri, (-5, 5, -5, 5), [O.BC_PERIODIC] * 4)
        M = O.Mesh.tri(xy, tri, tags, period)
        S = O.Solver(M)
        S.set_state(M.project(ex(M.quad_points(), 0.0)))
        S.advance(0.5)
        errs.append(H.l2_error(S, R, lambda x: ex(x, 0.5)))
    assert order(errs)[-1] > 2.2, errs


def test_e3_near_vacuum_advection_cartesian():
    """The paper's smooth near-vacuum test (Sec. 4.3.1) at a short final time: the limiters are on,
    positivity holds, and the error falls at a rate near 3."""
    R = O.RefElem(O.QUAD)
    T = 0.002
    errs = []
    for n in [12, 24, 48]:
        M = O.Mesh.cart(n, n, 0, 1, 0, 1, [O.BC_PERIODIC] * 4)
        S = O.Solver(M)
        S.set_state(M.project(H.cons(H.e3_prim(*np.moveaxis(M.quad_points(), -1, 0), 0.0))))
        S.advance(T)
        errs.append(H.l2_error(S, R, lambda x: H.cons(H.e3_prim(x[..., 0], x[..., 1], T))))
    assert order(errs)[-1] > 2.5, errs


@pytest.mark.parametrize("mesh_kind", ["cart", "tri", "line"])
def test_conservation_to_roundoff(mesh_kind):
    if mesh_kind == "cart":
        M = O.Mesh.cart(12, 10, 0, 1, 0, 1, [O.BC_PERIODIC] * 4)
    elif mesh_kind == "line":
        M = O.Mesh.line(40, 0, 1, O.BC_PERIODIC, O.BC_PERIODIC)
    else:
        xy, tri = I.lattice_delaunay(12, 5, periodic=True)
        M = O.Mesh.tri(xy, tri, I.boundary_tags(xy, tri, (0, 1, 0, 1), [O.BC_PERIODIC] * 4), (1.0, 1.0))
    Q = I.random_modal_state(M.N, M.dim, M.ML, seed=2, amp=0.5, rough_frac=0.2, rough_amp=3.0, p_range=(1e-5, 1.0))
    S = O.Solver(M)
    S.set_state(Q)
    tot0 = np.sum(Q[:, :, 0] * M.area[:, None], axis=0)
    for _ in range(10):
        S.step()
    Qn, _ = S.get_state()
    tot = np.sum(Qn[:, :, 0] * M.area[:, None], axis=0)
    scale = np.sum(np.abs(Q[:, :, 0]) * M.area[:, None], axis=0)
    assert np.all(np.abs(tot - tot0) <= 1e-13 * scale), (tot - tot0) / scale


def limited_point_values(S, R):
    pts = np.concatenate([R.xi_int, R.xi_edge.reshape(-1, R.dim)], 0)
    Q = S.stage(O.STAGE_QLIM)
    Phi = np.array([[R.phi(l, p) for l in range(R.ML)] for p in pts])
    return np.einsum("pl,nvl->npv", Phi, Q), Q[:, :, 0]


def test_positivity_sedov_cartesian():
    """Near-vacuum blast (the Cartesian stand-in of Sec. 4.3.2): p = 1e-10 background.  Every step:
    cell averages positive; after the moment limiter rho >= eps0 and p >= min(eps0, p_bar) at every
    quadrature point used by the update (Sec. 3.1)."""
    n = 16
    R = O.RefElem(O.QUAD)
    M = O.Mesh.cart(n, n, -1, 1, -1, 1, [O.BC_PERIODIC] * 4)
    S = O.Solver(M)
    S.set_state(I.sedov_cart_state(n, n))
    n_lim = 0
    for _ in range(40):
        S.step()
        q, qbar = limited_point_values(S, R)
        pbar = H.pressure(qbar)
        assert np.all(qbar[:, 0] > 0) and np.all(pbar > 0)
        assert np.all(q[..., 0] >= 1e-12 * (1 - 1e-9))
        assert np.all(H.pressure(q) >= np.minimum(1e-12, pbar)[:, None] * (1 - 1e-6) - 1e-16)
        n_lim += np.sum(S.stage(O.STAGE_THETA_MOM) < 1)
    Qn, _ = S.get_state()
    assert np.all(Qn[:, 0, 0] > 0) and np.all(H.pressure(Qn[:, :, 0]) > 0)
    assert n_lim > 0


def test_positivity_double_rarefaction_1d():
    """The double-rarefaction problem of Sec. 4.2.1 at Delta x = 1/100 (domain [0, 1], jump at 0.5,
    to t = 0.1): near-vacuum forms and every step stays positive."""
    n = 100
    M = O.Mesh.line(n, 0, 1, O.BC_TRANSPARENT, O.BC_TRANSPARENT)
    xc = (np.arange(n) + 0.5) / n
    prim = np.where((xc < 0.5)[:, None], [7, -1, 0.2], [7, 1, 0.2])
    S = O.Solver(M)
    S.set_state(I.averages_to_modal(I.prim_to_cons(prim, 1.4), 3))
    R = O.RefElem(O.LINE)
    while S.get_state()[1] < 0.1:
        S.step(0.1)
        q, qbar = limited_point_values(S, R)
        assert np.all(qbar[:, 0] > 0) and np.all(H.pressure(qbar) > 0)
        assert np.all(q[..., 0] >= 1e-12 * (1 - 1e-9))
    Qn, t = S.get_state()
    assert t == pytest.approx(0.1, abs=1e-15)
    assert Qn[:, 0, 0].min() < 0.5


def test_positivity_sedov_1d():
    """1D Sedov blast (Sec. 4.2.2): E = 3.2e6/dx in the centre cell, 1e-12 elsewhere, dx = 1/100."""
    n = 101
    M = O.Mesh.line(n, -0.5, 0.5, O.BC_TRANSPARENT, O.BC_TRANSPARENT)
    dx = 1.0 / n
    avg = np.zeros((n, 3))
    avg[:, 0] = 1.0
    avg[:, 2] = 1e-12
    avg[n // 2, 2] = 3200000.0 / dx
    S = O.Solver(M)
    S.set_state(I.averages_to_modal(avg, 3))
    for _ in range(30):
        S.step()
    Qn, _ = S.get_state()
    assert np.all(Qn[:, 0, 0] > 0) and np.all(H.pressure(Qn[:, :, 0]) > 0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_riemann_1d_against_exact(seed):
    """Seeded 1D Riemann problems (rho, p in U[0.1, 1], u in U[-1, 1]) on [0, 1] to t = 0.2: the L1
    density error against the exact solution falls under refinement and is small."""
    left, right = I.riemann_1d_params(seed)
    ex = ExactRiemann(left, right)
    errs = []
    for n in [50, 100, 200]:
        M = O.Mesh.line(n, 0, 1, O.BC_TRANSPARENT, O.BC_TRANSPARENT)
        S = O.Solver(M, cfl=0.1)
        S.set_state(I.riemann_1d_state(n, seed))
        S.advance(0.2)
        Q, t = S.get_state()
        exa = ex.cell_averages(0, 1, n, 0.2, 0.5, sub=8)
        errs.append(np.mean(np.abs(Q[:, 0, 0] - exa[:, 0])))
    assert errs[2] < errs[0]
    assert errs[2] < 0.02, errs


def test_reflective_wall_mirror_symmetry():
    """A reflective wall is equivalent to a mirror-image domain: a 1D problem on [0, 1] with a
    reflective right wall equals the left half of the mirrored problem on [0, 2] (Sec. 2.4)."""
    n = 40
    left, right = I.riemann_1d_params(3)
    xc = (np.arange(n) + 0.5) / n
    prim = np.where((xc < 0.4)[:, None], list(left), list(right))
    Qh = I.averages_to_modal(I.prim_to_cons(prim, 1.4), 3)
    Mh = O.Mesh.line(n, 0, 1, O.BC_TRANSPARENT, O.BC_REFLECTIVE)
    Sh = O.Solver(Mh, cfl=0.1)
    Sh.set_state(Qh)
    Qf = np.concatenate([Qh, Qh[::-1] * np.array([1, -1, 1])[None, :, None] * np.array([1, -1, 1])[None, None, :]], 0)
    Mf = O.Mesh.line(2 * n, 0, 2, O.BC_TRANSPARENT, O.BC_TRANSPARENT)
    Sf = O.Solver(Mf, cfl=0.1)
    Sf.set_state(Qf)
    for _ in range(20):
        Sh.step()
        Sf.step()
    a, _ = Sh.get_state()
    b, _ = Sf.get_state()
    assert np.allclose(a, b[:n], rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("axis", ["x", "y"])
def test_masked_cells_act_as_walls(axis):
    """Removed cells of a masked Cartesian mesh turn their neighbours' faces into boundaries of the
    given type: a 2n x m box whose upper half (in x or in y) is removed runs bit for bit like the
    n x m box with a reflective wall on that side (same cell order, same coordinates)."""
    n, m = 10, 7
    if axis == "x":
        keep = (np.arange(2 * n)[None, :] < n) & np.ones((m, 1), bool)
        Mm = O.Mesh.cart(2 * n, m, 0, 2, 0, 1, [O.BC_TRANSPARENT, O.BC_TRANSPARENT, O.BC_PERIODIC, O.BC_PERIODIC],
                         keep=keep, wall_bc=O.BC_REFLECTIVE)
        Mp = O.Mesh.cart(n, m, 0, 1, 0, 1, [O.BC_TRANSPARENT, O.BC_REFLECTIVE, O.BC_PERIODIC, O.BC_PERIODIC])
    else:
        keep = (np.arange(2 * m)[:, None] < m) & np.ones((1, n), bool)
        Mm = O.Mesh.cart(n, 2 * m, 0, 1, 0, 2, [O.BC_PERIODIC, O.BC_PERIODIC, O.BC_TRANSPARENT, O.BC_TRANSPARENT],
                         keep=keep, wall_bc=O.BC_REFLECTIVE)
        Mp = O.Mesh.cart(n, m, 0, 1, 0, 1, [O.BC_PERIODIC, O.BC_PERIODIC, O.BC_TRANSPARENT, O.BC_REFLECTIVE])
    assert (Mm.N, Mm.E) == (Mp.N, Mp.E) == (n * m, Mp.E)
    Q = I.random_modal_state(n * m, 2, 9, seed=11, amp=0.3, rough_frac=0.1, rough_amp=2.0, p_range=(1e-3, 1.0))
    out = []
    for M in (Mm, Mp):
        S = O.Solver(M)
        S.set_state(Q)
        for _ in range(5):
            S.step()
        out.append(S.get_state())
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]


def test_masked_walls_conserve_mass_and_energy():
    """A periodic box with a block of cells removed (reflective faces) and a notch across the
    periodic seam: mass and energy stay constant to round-off over ten steps (no mass or energy
    crosses a reflective face), while the x-momentum does not (the walls push), and a uniform
    flow stays uniform except next to the walls after one step (every other cell sees the same
    flux on opposite faces)."""
    nx, ny = 24, 20
    keep = np.ones((ny, nx), bool)
    keep[7:12, 9:15] = False        # block
    keep[3:6, 0:2] = False          # notch at the x-low side: its x-high partner faces it periodically
    M = O.Mesh.cart(nx, ny, 0, 2.4, 0, 2.0, [O.BC_PERIODIC] * 4, keep=keep, wall_bc=O.BC_REFLECTIVE)
    assert M.N == keep.sum() and M.area.sum() == pytest.approx(2.4 * 2.0 * keep.mean(), rel=1e-13)
    Q = I.random_modal_state(M.N, 2, 9, seed=12, amp=0.5, rough_frac=0.2, rough_amp=3.0, p_range=(1e-5, 1.0))
    mx = Q[:, 1, 0] + 0.5 * Q[:, 0, 0]  # a mean flow into the walls, pressure unchanged
    Q[:, 3, 0] += 0.5 * (mx**2 - Q[:, 1, 0] ** 2) / Q[:, 0, 0]
    Q[:, 1, 0] = mx
    S = O.Solver(M)
    S.set_state(Q)
    tot0 = np.sum(Q[:, :, 0] * M.area[:, None], axis=0)
    for _ in range(10):
        S.step()
    Qn, _ = S.get_state()
    tot = np.sum(Qn[:, :, 0] * M.area[:, None], axis=0)
    scale = np.sum(np.abs(Q[:, :, 0]) * M.area[:, None], axis=0)
    assert abs(tot[0] - tot0[0]) <= 1e-13 * scale[0] and abs(tot[3] - tot0[3]) <= 1e-13 * scale[3]
    assert abs(tot[1] - tot0[1]) > 1e-6 * scale[1]
    # uniform flow: one step changes only the cells with a face on a removed cell
    U = I.averages_to_modal(I.prim_to_cons(np.tile([1.0, 0.7, 0.4, 1.0], (M.N, 1)), 1.4), 9)
    S = O.Solver(M)
    S.set_state(U)
    S.step()
    Un, _ = S.get_state()
    changed = np.abs(Un[:, :, 0] - U[:, :, 0]).max(axis=1) > 1e-12
    ids = -np.ones(nx * ny, int)
    ids[keep.ravel()] = np.arange(M.N)
    jj, ii = np.nonzero(keep)
    walled = np.zeros(M.N, bool)
    for dj, di in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        walled |= ~keep[(jj + dj) % ny, (ii + di) % nx]
    assert np.array_equal(changed[ids[keep.ravel()]], walled)


@pytest.mark.parametrize("mesh_kind", ["line", "cart", "tri"])
def test_wave_speed_from_averages(mesh_kind):
    """With the wave speed taken over the cell averages only, s is the largest |u| + c of the
    averages and dt = CFL / (s max_i |dT_i| / (2 |T_i|)) (|dT_i| = 2 in 1D, where the factor is
    1/dx), recomputed here from the state and the mesh; and s never exceeds the default s, which
    also takes the limited points."""
    if mesh_kind == "cart":
        M = O.Mesh.cart(12, 10, 0, 1.2, 0, 1, [O.BC_PERIODIC] * 4)
    elif mesh_kind == "line":
        M = O.Mesh.line(40, 0, 1, O.BC_TRANSPARENT, O.BC_TRANSPARENT)
    else:
        M = O.Mesh.tri(*I.lattice_delaunay(12, 5))
    Q = I.random_modal_state(M.N, M.dim, M.ML, seed=4, amp=0.5, rough_frac=0.2, rough_amp=3.0, p_range=(1e-5, 1.0))
    A = O.Solver(M, s_from_averages=True)
    A.set_state(Q)
    A.step()
    s_a, dt_a = A.stage(O.STAGE_SDT)
    q = Q[:, :, 0]
    speed = np.hypot.reduce(q[:, 1:-1] / q[:, :1], axis=1) if M.dim == 2 else np.abs(q[:, 1] / q[:, 0])
    speed = speed + np.sqrt(1.4 * H.pressure(q) / q[:, 0])
    assert s_a == pytest.approx(speed.max(), rel=1e-13)
    geo = (M.perim / (2 * M.area)).max() if M.dim == 2 else (1.0 / M.area).max()
    assert dt_a == pytest.approx(0.08 / (s_a * geo), rel=1e-13)
    B = O.Solver(M)
    B.set_state(Q)
    B.step()
    assert B.stage(O.STAGE_SDT)[0] >= s_a
