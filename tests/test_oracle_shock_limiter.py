"""Pins of the oracle's shock-capturing limiter (Sec. 1.5 Step 5, Sec. 4.1).

The paper cites this limiter without defining it; the oracle's reading works on the primitive
variables w in (rho, u[, v], p) of each cell: bounds
    M_w = max(w_bar_i + delta_i, max_j w_bar_j),   m_w = min(w_bar_i - delta_i, min_j w_bar_j)
over the edge neighbours j (their averages after the update, the boundary operator's state across a
boundary edge), delta_i = alpha0 h_i^1.5 with h_i = dx (1D), sqrt|T_i| (quadrilaterals) and
sqrt(2|T_i|) (triangles); one factor theta scales every mode l >= 2, the largest factor for which the
deviation of each primitive variable from w_bar_i, scaled linearly by theta, stays within the
bounds at every limiter point (velocity and pressure sampled where the density is positive).

What is pinned here, independently of the closed form the oracle evaluates:
 * cell averages are unchanged and theta is in [0, 1]; the higher modes are exactly theta times the
   updated ones;
 * density is linear in theta, so after limiting every point density lies within [m_rho, M_rho];
 * pressure is concave along theta (Sec. 3.1), so the linearly scaled lower bound is safe: every
   point with positive updated density has p >= m_p after limiting;
 * theta is maximal: it equals the largest factor found by bisection on the linearly scaled
   constraints;
 * where a variable is linear in theta (velocity in a cell of uniform density; pressure in a cell of
   uniform density and momentum) its bounds hold exactly after limiting and theta is the largest
   factor found by bisection on the limited state's actual values;
 * the neighbour bounds come from the averages after the update, not before it;
 * h_i equals the lattice spacing on a split-square triangle lattice, the cell size on quadrilaterals
   and dx in 1D;
 * a hand-computed three-cell 1D case.
For velocity in general and for the pressure's upper bound the reading's factor is a linearisation:
those bounds hold to first order in the deviation only (reading of the cited limiter).
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1601_08145_amd import inputs as I
from tests import helpers as H

G = 1.4


def points(kind):
    R = O.RefElem(kind)
    xi = np.vstack([R.xi_int, R.xi_edge.reshape(-1, R.dim)])
    Phi = np.array([[R.phi(l, x) for l in range(R.ML)] for x in xi])
    return R, Phi


def prim(q):
    dim = q.shape[-1] - 2
    w = np.empty_like(q)
    w[..., 0] = q[..., 0]
    with np.errstate(divide="ignore", invalid="ignore"):
        w[..., 1:1 + dim] = q[..., 1:1 + dim] / q[..., :1]
    w[..., -1] = H.pressure(q)
    return w


def at_points(Q, Phi):
    """q at the limiter points: (N, P, V)."""
    return np.einsum("nvl,pl->npv", Q, Phi)


def bounds(avg, nb, delta):
    """(m, M) per cell and primitive variable from the cell's own averages, its neighbours'
    (transparent boundary: the own average) and the relaxation delta."""
    wb = prim(avg)
    Mx = wb + delta[:, None]
    Mn = wb - delta[:, None]
    for k in range(nb.shape[1]):
        j = nb[:, k]
        wn = np.where((j >= 0)[:, None], wb[np.maximum(j, 0)], wb)
        Mx = np.maximum(Mx, wn)
        Mn = np.minimum(Mn, wn)
    return Mn, Mx


def bisect_linear(wb, wpt, valid, Mn, Mx, it=80):
    """Largest theta in [0, 1] with m <= wb + theta (w_m - wb) <= M at every point (valid mask per
    point and variable), by bisection."""
    def ok(th):
        w = wb[:, None, :] + th[:, None, None] * (wpt - wb[:, None, :])
        good = (w <= Mx[:, None, :]) & (w >= Mn[:, None, :])
        return np.all(good | ~valid, axis=(1, 2))

    lo = np.zeros(len(wb))
    hi = np.ones(len(wb))
    full = ok(hi)
    for _ in range(it):
        mid = 0.5 * (lo + hi)
        g = ok(mid)
        lo = np.where(g, mid, lo)
        hi = np.where(g, hi, mid)
    return np.where(full, 1.0, lo)


def mesh_case(kind, seed):
    if kind == "tri":
        xy, tri = I.lattice_delaunay(11, seed)
        M = O.Mesh.tri(xy, tri)
        _, area, nb = H.tri_geometry(xy, tri)
        h = np.sqrt(2 * area)
    elif kind == "cart":
        n = 9
        M = O.Mesh.cart(n, n, 0, 1, 0, 1, [O.BC_PERIODIC] * 4)
        N = n * n
        area = np.full(N, 1.0 / N)
        nb = np.zeros((N, 4), np.int64)
        for j in range(n):
            for i in range(n):
                nb[i + n * j] = [i + n * ((j - 1) % n), (i + 1) % n + n * j, i + n * ((j + 1) % n), (i - 1) % n + n * j]
        h = np.sqrt(area)
    else:
        n = 48
        M = O.Mesh.line(n, 0, 1, O.BC_PERIODIC, O.BC_PERIODIC)
        area = np.full(n, 1.0 / n)
        nb = np.stack([(np.arange(n) - 1) % n, (np.arange(n) + 1) % n], 1)
        h = area.copy()
    return M, nb, h


@pytest.mark.parametrize("kind", ["tri", "cart", "line"])
def test_shock_limiter_bounds_and_maximality_on_rough_states(kind):
    M, nb, h = mesh_case(kind, 3)
    kcode = {"tri": O.TRI, "cart": O.QUAD, "line": O.LINE}[kind]
    R, Phi = points(kcode)
    alpha0 = 0.4
    delta = alpha0 * h ** 1.5
    Q0 = I.random_modal_state(M.N, M.dim, M.ML, seed=11, amp=0.4, rough_frac=0.25, rough_amp=1.5,
                              p_range=(1e-3, 1.0))
    S = O.Solver(M, alpha0=alpha0)
    S.set_state(Q0)
    S.step()
    Qpre = S.stage(O.STAGE_QLIM)     # state at the start of the step
    Qu = S.stage(O.STAGE_QUPD)       # after the update: what the shock limiter sees
    th = S.stage(O.STAGE_THETA_SC)
    Qs, _ = S.get_state()            # after the shock limiter

    # averages unchanged, theta in [0, 1], higher modes scaled by exactly theta
    assert np.array_equal(Qs[:, :, 0], Qu[:, :, 0])
    assert np.all((th >= 0) & (th <= 1))
    lim = th < 1
    assert np.array_equal(Qs[~lim], Qu[~lim])
    assert np.array_equal(Qs[lim][:, :, 1:], th[lim][:, None, None] * Qu[lim][:, :, 1:])
    assert lim.sum() >= 5, lim.sum()

    avg = Qu[:, :, 0]
    Mn, Mx = bounds(avg, nb, delta)
    wb = prim(avg)
    qu = at_points(Qu, Phi)
    qs = at_points(Qs, Phi)
    V = M.V
    rho_pos = qu[..., 0] > 0
    valid = np.ones(qu.shape, bool)
    valid[..., 1:] = rho_pos[..., None]
    wu = prim(np.where(rho_pos[..., None], qu, 1.0))

    # density: linear in theta, both bounds hold after limiting
    tol = 1e-12
    rs = qs[..., 0]
    assert np.all(rs <= Mx[:, None, 0] + tol * np.abs(Mx[:, None, 0]) + 1e-15)
    assert np.all(rs >= Mn[:, None, 0] - tol * np.abs(Mn[:, None, 0]) - 1e-15)
    # pressure: concave along theta, the lower bound holds where the updated density was positive
    ps = H.pressure(np.where(rho_pos[..., None], qs, 1.0))
    assert np.all((ps >= Mn[:, None, V - 1] - 1e-12 * np.abs(Mn[:, None, V - 1]) - 1e-15) | ~rho_pos)

    # maximality: the bisection on the linearly scaled constraints gives the same factor
    tb = bisect_linear(wb, wu, valid, Mn, Mx)
    assert np.max(np.abs(tb - th)) <= 1e-12, np.max(np.abs(tb - th))

    # the pins discriminate: bounds from the averages before the update, or h = sqrt|T| on
    # triangles, or swapped bounds give other factors
    Mn0, Mx0 = bounds(Qpre[:, :, 0], nb, delta)
    assert np.max(np.abs(bisect_linear(wb, wu, valid, Mn0, Mx0) - th)) > 1e-6
    assert np.max(np.abs(bisect_linear(wb, wu, valid, 2 * wb - Mx, 2 * wb - Mn) - th)) > 1e-6
    if kind == "tri":
        Mn1, Mx1 = bounds(avg, nb, alpha0 * np.sqrt(h ** 2 / 2) ** 1.5)
        assert np.max(np.abs(bisect_linear(wb, wu, valid, Mn1, Mx1) - th)) > 1e-6
    # both kinds of bound bind somewhere: the relaxation and a neighbour's average
    hi_bind = (wu > Mx[:, None, :]) & valid
    relax = np.isclose(Mx, wb + delta[:, None], rtol=0, atol=1e-14)
    assert np.any(hi_bind & relax[:, None, :]) and np.any(hi_bind & ~relax[:, None, :])


def _linear_case(which, seed=5):
    """A triangle mesh whose cells deviate from their averages only through the variable(s) of
    `which`: 'rho' (momentum rho u0 and energy linear in rho, so velocity and pressure stay
    uniform), 'u' (uniform density, linear momentum, energy that keeps the pressure uniform at
    theta = 1 up to a small quadratic term), 'p' (uniform density and momentum).  The neighbours'
    averages spread by +-0.002 in the tested variable and by +-0.3 in the others, so that only the
    tested variable's bounds can bind."""
    xy, tri = I.lattice_delaunay(7, seed)
    M = O.Mesh.tri(xy, tri)
    _, area, nb = H.tri_geometry(xy, tri)
    N = M.N
    R, Phi = points(O.TRI)
    g = np.random.default_rng(seed)
    tested = {"rho": [0], "u": [1, 2], "p": [3]}[which]
    spread = np.array([0.002 if c in tested else 0.3 for c in range(4)])
    avg_prim = np.array([1.0, 0.3, -0.2, 1.0]) + g.uniform(-1, 1, (N, 4)) * spread
    Q = np.zeros((N, 4, 6))
    # project functions of the reference coordinates onto the basis with an independent rule
    pts, w = H.error_rule(O.TRI, 8)
    B = np.array([[R.phi(l, x) for l in range(6)] for x in pts])
    X, Y = pts[:, 0] - 1 / 3, pts[:, 1] - 1 / 3
    for i in range(N):
        r0, u0, v0, p0 = avg_prim[i]
        c = g.uniform(-1, 1, 5)
        lin = c[0] * X + c[1] * Y
        quad = lin + c[2] * X * X + c[3] * X * Y + c[4] * Y * Y
        one = np.ones_like(X)
        if which == "rho":
            rho = r0 * (1 + 0.3 * quad)
            q = H.cons(np.stack([rho, u0 * one, v0 * one, p0 * one], -1))
        elif which == "u":
            mx = r0 * (u0 + 0.05 * lin)
            my = r0 * (v0 - 0.04 * lin)
            E = p0 / (G - 1) + 0.5 * (mx * mx + my * my) / r0
            q = np.stack([r0 * one, mx, my, E], -1)
        else:
            E = p0 * (1 + 0.3 * quad) / (G - 1) + 0.5 * r0 * (u0 * u0 + v0 * v0)
            q = np.stack([r0 * one, r0 * u0 * one, r0 * v0 * one, E], -1)
        Q[i] = np.einsum("pv,p,pl->vl", q, w, B)
        Q[i, :, 0] = H.cons(avg_prim[i])  # the average state exactly as chosen
    return M, nb, np.sqrt(2 * area), Q, Phi


@pytest.mark.parametrize("which", ["rho", "u", "p"])
def test_shock_limiter_exact_where_variable_is_linear(which):
    """Where a primitive variable is linear in theta its bounds hold exactly after limiting, and
    theta is the largest factor with the limited state's actual values inside the bounds."""
    M, nb, h, Q, Phi = _linear_case(which)
    alpha0 = 0.05
    delta = alpha0 * h ** 1.5
    S = O.Solver(M, alpha0=alpha0)
    Mn, Mx = bounds(Q[:, :, 0], nb, delta)
    var = {"rho": [0], "u": [1, 2], "p": [3]}[which]
    n_lim = 0
    for i in range(M.N):
        th, Qi = S.shock_limit(Q, i)
        assert 0 <= th <= 1
        assert np.array_equal(Qi[:, 0], Q[i, :, 0])
        w = prim(np.einsum("vl,pl->pv", Qi, Phi))
        for c in var:
            assert np.all(w[:, c] <= Mx[i, c] + 1e-13) and np.all(w[:, c] >= Mn[i, c] - 1e-13), (i, c)

        def inside(t):
            Qt = Q[i].copy()
            Qt[:, 1:] *= t
            wt = prim(np.einsum("vl,pl->pv", Qt, Phi))
            return all(np.all(wt[:, c] <= Mx[i, c]) and np.all(wt[:, c] >= Mn[i, c]) for c in range(4))

        if inside(1.0):
            assert th == 1.0
            continue
        n_lim += 1
        lo, hi = 0.0, 1.0
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            lo, hi = (mid, hi) if inside(mid) else (lo, mid)
        assert abs(th - lo) <= 1e-11, (i, th, lo)
    assert n_lim >= M.N // 3, n_lim


@pytest.mark.parametrize("kind", ["tri", "cart", "line", "tet"])
def test_shock_limiter_relaxation_uses_cell_size(kind):
    """delta = alpha0 h^1.5 with h the lattice spacing of a split-square triangle lattice
    (h = sqrt(2|T|)), the side of a square cell (sqrt|T|), dx in 1D and the lattice spacing of a
    cube split into six tetrahedra (h = cbrt(6|T|)): a cell whose neighbours all share its average
    is bound by the relaxation alone, theta = delta / max_m |rho_m - rho_bar|."""
    n = 6
    if kind == "tet":
        n = 3
        xyz, tet = I.lattice_tets(n + 1, 0, jitter=0.0)
        M = O.Mesh.tet(xyz, tet)
        kcode, hlat = O.TET, 1.0 / n
    elif kind == "tri":
        xy, tri = I.lattice_delaunay(n + 1, 0, jitter=0.0)
        M = O.Mesh.tri(xy, tri)
        kcode, hlat = O.TRI, 1.0 / n
    elif kind == "cart":
        M = O.Mesh.cart(n, n, 0, 1, 0, 1, [O.BC_PERIODIC] * 4)
        kcode, hlat = O.QUAD, 1.0 / n
    else:
        M = O.Mesh.line(n, 0, 2, O.BC_PERIODIC, O.BC_PERIODIC)
        kcode, hlat = O.LINE, 2.0 / n
    R, Phi = points(kcode)
    alpha0 = 0.07
    Q = np.zeros((M.N, M.V, M.ML))
    Q[:, :, 0] = H.cons(np.array([1.0] + [0.0] * M.dim + [1.0])[None, :].repeat(M.N, 0))
    i = M.N // 2
    # a density deviation in the second mode only, with the momentum zero and the energy uniform
    # (velocity 0 and pressure 1 everywhere)
    Q[i, 0, 1] = 0.3
    dev = np.max(np.abs(np.einsum("l,pl->p", Q[i, 0], Phi) - 1.0))
    th, _ = O.Solver(M, alpha0=alpha0).shock_limit(Q, i)
    expect = alpha0 * hlat ** 1.5 / dev
    assert 0 < expect < 1
    assert abs(th - expect) <= 1e-13 * expect, (th, expect)


def test_shock_limiter_three_cells_by_hand():
    """1D, three periodic cells of width 1/3.  Middle cell: rho = 1 + 0.2 xi (xi in [-1, 1]; the
    mode-2 coefficient 0.2/sqrt(3) of the orthonormal sqrt(3) xi), momentum 0, E = 2.5 (p = 1).
    Left neighbour's average density 1.05, right 0.9, both at rest with p = 1; delta = 0.01.
    Bounds on rho: M = max(1.01, 1.05, 0.9) = 1.05, m = min(0.99, 1.05, 0.9) = 0.9.  The extremes
    1.2 and 0.8 (at the cell's ends, which are limiter points) give (1.05 - 1)/(1.2 - 1) = 0.25
    and (1 - 0.9)/(1 - 0.8) = 0.5; velocity and pressure are uniform: theta = 0.25.  With the
    relaxation alone binding (both neighbours at density 1): theta = 0.01/0.2 = 0.05."""
    dx = 1.0 / 3.0
    M = O.Mesh.line(3, 0, 1, O.BC_PERIODIC, O.BC_PERIODIC)
    S = O.Solver(M, alpha0=0.01 / dx ** 1.5)
    Q = np.zeros((3, 3, 3))
    for c, r in enumerate([1.05, 1.0, 0.9]):
        Q[c, :, 0] = [r, 0.0, 2.5]
    Q[1, 0, 1] = 0.2 / math.sqrt(3.0)
    th, Qi = S.shock_limit(Q, 1)
    assert abs(th - 0.25) <= 1e-14, th
    assert np.allclose(Qi[0], [1.0, 0.25 * 0.2 / math.sqrt(3.0), 0.0], rtol=0, atol=1e-16)
    Q[0, 0, 0] = Q[2, 0, 0] = 1.0
    th, _ = S.shock_limit(Q, 1)
    assert abs(th - 0.05) <= 1e-14, th
