"""Seeded synthetic inputs: meshes and initial states.

This module holds none of the DG method's arithmetic (no basis, quadrature, flux or limiter):
it draws random numbers and builds meshes and initial conserved states of the shapes used in
the paper's experiments (Sec. 4) and in the benchmark workloads.  Both the GPU library's tests
and benchmark and the oracle's tests take their inputs from here, so that the two sides receive
identical arrays.

Array conventions (the library's public layout):
  * triangle meshes: node coordinates xy[n_nodes][2], counter-clockwise triangles tri[n_tri][3];
  * initial states: modal coefficients Q[n_elem][n_var][n_modes] (float64), conserved variables
    (rho, M, E) in 1D and (rho, Mx, My, E) in 2D.  Piecewise-constant states carry only mode 1
    (the cell average, since the first basis function is identically one).
"""
import math

import numpy as np

from scipy.spatial import Delaunay

# Boundary-condition codes shared with the public interface (include/lxw.h).
BC_PERIODIC, BC_TRANSPARENT, BC_REFLECTIVE, BC_INFLOW = 0, 1, 2, 3


def rng(seed):
    return np.random.default_rng(np.random.SeedSequence(int(seed)))


# ---------------------------------------------------------------------------------------------
# Meshes
# ---------------------------------------------------------------------------------------------

def lattice_delaunay(n, seed, jitter=0.3, box=(0.0, 1.0, 0.0, 1.0), periodic=False):
    """Delaunay triangulation of an n x n lattice of points on `box`, with interior points
    jittered by U[-jitter*h, jitter*h]^2 (h = lattice spacing), boundary points jittered only
    along their boundary line and corners fixed.  With periodic=True the jitter of the points on
    the x-high / y-high sides copies that of their x-low / y-low partners, so that boundary edges
    pair up under translation by one period.

    Returns (xy[n*n][2], tri[n_tri][3]) with counter-clockwise triangles; n_tri = 2(n-1)^2 for a
    point set whose boundary points are all on the hull."""
    x0, x1, y0, y1 = box
    hx = (x1 - x0) / (n - 1)
    hy = (y1 - y0) / (n - 1)
    g = rng(seed)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    dx = g.uniform(-jitter * hx, jitter * hx, size=i.shape)
    dy = g.uniform(-jitter * hy, jitter * hy, size=i.shape)
    bx = (i == 0) | (i == n - 1)
    by = (j == 0) | (j == n - 1)
    dx[bx] = 0.0
    dy[by] = 0.0
    if periodic:
        dy[n - 1, :] = dy[0, :]
        dx[:, n - 1] = dx[:, 0]
    x = x0 + i * hx + dx
    y = y0 + j * hy + dy
    xy = np.stack([x.ravel(), y.ravel()], axis=1)
    tri = Delaunay(xy).simplices.astype(np.int32)
    a = xy[tri]
    cross = (a[:, 1, 0] - a[:, 0, 0]) * (a[:, 2, 1] - a[:, 0, 1]) - (a[:, 1, 1] - a[:, 0, 1]) * (a[:, 2, 0] - a[:, 0, 0])
    flip = cross < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    return np.ascontiguousarray(xy), np.ascontiguousarray(tri)


def boundary_tags(xy, tri, box, codes):
    """Per triangle edge (n_tri x 3; edge k joins vertices k and k+1) the boundary code of the
    side of `box` the edge lies on (codes = {x-low, x-high, y-low, y-high}), -1 elsewhere."""
    x0, x1, y0, y1 = box
    tol = 1e-9 * max(x1 - x0, y1 - y0)
    tags = np.full(tri.shape, -1, np.int32)
    for k in range(3):
        a = xy[tri[:, k]]
        b = xy[tri[:, (k + 1) % 3]]
        for side, (coord, val) in enumerate([(0, x0), (0, x1), (1, y0), (1, y1)]):
            on = (np.abs(a[:, coord] - val) < tol) & (np.abs(b[:, coord] - val) < tol)
            tags[on, k] = codes[side]
    return tags


def lattice_tets(n, seed, jitter=0.12, box=(0.0, 1.0, 0.0, 1.0, 0.0, 1.0), periodic=False):
    """Tetrahedral mesh of an n x n x n lattice of points on `box`: each lattice cube split into
    the six tetrahedra along its main diagonal (the Kuhn subdivision, conforming across cubes),
    interior points jittered by U[-jitter*h, jitter*h]^3, points on a side jittered only within
    it.  With periodic=True the points on the high sides copy the jitter of their low-side
    partners, so that boundary faces pair up under translation by one period.

    Returns (xyz[n^3][3], tet[6 (n-1)^3][4]) with positively oriented tetrahedra."""
    x0, x1, y0, y1, z0, z1 = box
    h = np.array([(x1 - x0), (y1 - y0), (z1 - z0)]) / (n - 1)
    g = rng(seed)
    idx = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), -1)  # [i][j][k][3]
    d = g.uniform(-jitter, jitter, size=idx.shape) * h
    for a in range(3):
        on = (idx[..., a] == 0) | (idx[..., a] == n - 1)
        d[..., a][on] = 0.0
    if periodic:
        d[n - 1, :, :] = d[0, :, :]
        d[:, n - 1, :] = d[:, 0, :]
        d[:, :, n - 1] = d[:, :, 0]
    xyz = (np.array([x0, y0, z0]) + idx * h + d).reshape(-1, 3)
    node = lambda i, j, k: (i * n + j) * n + k
    c = np.stack(np.meshgrid(np.arange(n - 1), np.arange(n - 1), np.arange(n - 1), indexing="ij"), -1).reshape(-1, 3)
    tets = []
    for perm in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
        v = [c.copy()]
        for a in perm:
            nxt = v[-1].copy()
            nxt[:, a] += 1
            v.append(nxt)
        tets.append(np.stack([node(w[:, 0], w[:, 1], w[:, 2]) for w in v], 1))
    tet = np.concatenate(tets, 0).astype(np.int32)
    a = xyz[tet]
    vol = np.einsum("ij,ij->i", a[:, 1] - a[:, 0], np.cross(a[:, 2] - a[:, 0], a[:, 3] - a[:, 0]))
    flip = vol < 0
    tet[flip] = tet[flip][:, [0, 2, 1, 3]]
    return np.ascontiguousarray(xyz), np.ascontiguousarray(tet)


TET_FACES = ((1, 2, 3), (0, 3, 2), (0, 1, 3), (0, 2, 1))  # face k opposite vertex k, outward


def boundary_tags_tet(xyz, tet, box, codes):
    """Per tetrahedron face (n_tet x 4; face k opposite vertex k) the boundary code of the side of
    `box` the face lies on (codes = {x-low, x-high, y-low, y-high, z-low, z-high}), -1 elsewhere."""
    tol = 1e-9 * max(box[1] - box[0], box[3] - box[2], box[5] - box[4])
    tags = np.full(tet.shape, -1, np.int32)
    for k, f in enumerate(TET_FACES):
        p = xyz[tet[:, list(f)]]  # [n][3][3]
        for side in range(6):
            a, val = side // 2, box[side]
            on = np.all(np.abs(p[:, :, a] - val) < tol, axis=1)
            tags[on, k] = codes[side]
    return tags


def ramp_channel(n_target, seed, angle_deg=30.0, length=4.0, height=1.5, ramp_x=0.5, ramp_len=1.0, jitter=0.25):
    """Channel [0, length] x [floor, height] whose floor rises at `angle_deg` from x = ramp_x over a
    horizontal run ramp_len and is flat after it (a double-Mach-reflection shaped domain), meshed
    by Delaunay triangulation of a jittered point lattice that follows the floor.  Returns
    (xy, tri, tags) with tags per triangle edge (edge k joins vertices k and k+1): 0 on the inflow
    side x = 0, 1 on the outflow side x = length, 3 on the top, 2 (wall) on the floor and the ramp,
    -1 for interior edges."""
    g = rng(seed)
    ta = math.tan(math.radians(angle_deg))

    def floor(x):
        return np.clip(x - ramp_x, 0.0, ramp_len) * ta

    xs = np.linspace(0.0, length, 20001)
    area = np.trapezoid(height - floor(xs), xs)
    n_pts = n_target / 2.0
    ny = max(3, int(round(math.sqrt(n_pts * height / length))) + 1)
    nx = max(3, int(round(n_pts / ny)) + 1)
    s = np.linspace(0.0, length, nx)
    r = np.linspace(0.0, 1.0, ny)
    S, Rr = np.meshgrid(s, r, indexing="ij")
    fl = floor(S)
    hx = length / (nx - 1)
    dxj = g.uniform(-jitter * hx, jitter * hx, size=S.shape)
    dyj = g.uniform(-jitter, jitter, size=S.shape) / (ny - 1)
    dxj[0, :] = dxj[-1, :] = 0.0
    dxj[:, 0] = dxj[:, -1] = 0.0   # floor and top points keep their x (the floor has a kink)
    dyj[:, 0] = dyj[:, -1] = 0.0
    X = S + dxj
    Y = floor(X) + np.clip(Rr + dyj, 0.0, 1.0) * (height - floor(X))
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    tri = Delaunay(xy).simplices.astype(np.int32)
    a = xy[tri]
    c = a.mean(axis=1)
    tri = tri[c[:, 1] > floor(c[:, 0]) + 1e-12]  # the hull bridges the concave ramp foot
    a = xy[tri]
    cross = (a[:, 1, 0] - a[:, 0, 0]) * (a[:, 2, 1] - a[:, 0, 1]) - (a[:, 1, 1] - a[:, 0, 1]) * (a[:, 2, 0] - a[:, 0, 0])
    flip = cross < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    tri = np.ascontiguousarray(tri)
    # boundary edges: those used by one triangle only
    e = np.concatenate([np.sort(np.stack([tri[:, k], tri[:, (k + 1) % 3]], 1), 1) for k in range(3)], 0)
    key = e[:, 0].astype(np.int64) * len(xy) + e[:, 1]
    uniq, inv, cnt = np.unique(key, return_inverse=True, return_counts=True)
    on_bnd = (cnt[inv] == 1).reshape(3, -1).T  # n_tri x 3
    tags = np.full(tri.shape, -1, np.int32)
    tol = 1e-9
    for k in range(3):
        pa = xy[tri[:, k]]
        pb = xy[tri[:, (k + 1) % 3]]
        t = np.full(len(tri), 2, np.int32)
        t[(np.abs(pa[:, 0]) < tol) & (np.abs(pb[:, 0]) < tol)] = 0
        t[(np.abs(pa[:, 0] - length) < tol) & (np.abs(pb[:, 0] - length) < tol)] = 1
        t[(np.abs(pa[:, 1] - height) < tol) & (np.abs(pb[:, 1] - height) < tol)] = 3
        tags[on_bnd[:, k], k] = t[on_bnd[:, k]]
    return np.ascontiguousarray(xy), tri, tags


# Shock-diffraction domains of Sec. 4 (the block step and the 120-degree wedge).  Both are the box
# [0, 13] x [0, 11] minus a solid: the step removes [0, 1] x [0, 6]; the wedge removes the triangle
# (0, 0), (0, 6), (3.4, 6), whose slanted face and the top y = 6 meet at an angle of about 120
# degrees.  The gas enters above the solid (x = 0, 6 <= y <= 11); the solid's surface is a wall;
# every other side is transparent.
DIFFRACTION = {
    "step": {"solid": [(0.0, 0.0), (1.0, 0.0), (1.0, 6.0), (0.0, 6.0)], "x_shock": 1.0, "mach": 5.09, "t_end": 2.3},
    "wedge": {"solid": [(0.0, 0.0), (3.4, 6.0), (0.0, 6.0)], "x_shock": 3.4, "mach": 10.0, "t_end": 0.9},
}


def _in_polygon(pts, poly):
    """Points strictly inside a convex polygon given counter-clockwise (margin 1e-9)."""
    inside = np.ones(len(pts), dtype=bool)
    for k in range(len(poly)):
        (ax, ay), (bx, by) = poly[k], poly[(k + 1) % len(poly)]
        inside &= (bx - ax) * (pts[:, 1] - ay) - (by - ay) * (pts[:, 0] - ax) > 1e-9
    return inside


def _dist_to_polygon_edges(pts, poly):
    d = np.full(len(pts), np.inf)
    for k in range(len(poly)):
        a, b = np.array(poly[k]), np.array(poly[(k + 1) % len(poly)])
        ab = b - a
        t = np.clip(((pts - a) @ ab) / (ab @ ab), 0.0, 1.0)
        d = np.minimum(d, np.linalg.norm(pts - (a + t[:, None] * ab), axis=1))
    return d


def diffraction_domain(kind, n_target, seed, jitter=0.25, box=(13.0, 11.0)):
    """Triangle mesh of the `kind` ("step" or "wedge") shock-diffraction domain with about n_target
    triangles: a jittered lattice of spacing h, the solid's points removed, points placed every
    about h along the solid's surface (lattice points closer than 0.55 h to it dropped), Delaunay
    triangulation, triangles inside the solid removed.  Returns (xy, tri, tags) with tags per
    triangle edge (edge k joins vertices k and k+1): 0 on the inflow side (x = 0 above the solid),
    2 on the solid's surface, 1 on the other sides, -1 for interior edges."""
    spec = DIFFRACTION[kind]
    solid = spec["solid"]
    W, H = box
    sx, sy = np.array(solid).T
    solid_area = 0.5 * abs(np.dot(sx, np.roll(sy, -1)) - np.dot(sy, np.roll(sx, -1)))
    area = W * H - solid_area
    h = math.sqrt(2.0 * area / n_target)
    g = rng(seed)
    nx, ny = int(round(W / h)) + 1, int(round(H / h)) + 1
    X, Y = np.meshgrid(np.linspace(0.0, W, nx), np.linspace(0.0, H, ny), indexing="ij")
    hx, hy = W / (nx - 1), H / (ny - 1)
    dx = g.uniform(-jitter * hx, jitter * hx, X.shape)
    dy = g.uniform(-jitter * hy, jitter * hy, X.shape)
    dx[0, :] = dx[-1, :] = 0.0
    dy[:, 0] = dy[:, -1] = 0.0
    dx[:, 0] = dx[:, -1] = 0.0
    dy[0, :] = dy[-1, :] = 0.0
    pts = np.stack([(X + dx).ravel(), (Y + dy).ravel()], axis=1)
    keep = ~_in_polygon(pts, solid) & (_dist_to_polygon_edges(pts, solid) > 0.55 * min(hx, hy))
    pts = pts[keep]
    # points along the solid's surface (its edges that lie inside the box), spacing about h
    surf = []
    for k in range(len(solid)):
        a, b = np.array(solid[k]), np.array(solid[(k + 1) % len(solid)])
        if (a[0] == 0.0 and b[0] == 0.0) or (a[1] == 0.0 and b[1] == 0.0):
            continue  # on the box boundary: the solid's back, not in contact with the gas
        m = max(1, int(round(np.linalg.norm(b - a) / min(hx, hy))))
        surf.append(a[None, :] + np.linspace(0.0, 1.0, m + 1)[:, None] * (b - a)[None, :])
    surf = np.concatenate(surf)
    xy = np.concatenate([pts, surf])
    xy = np.unique(np.round(xy, 12), axis=0)
    tri = Delaunay(xy).simplices.astype(np.int32)
    c = xy[tri].mean(axis=1)
    tri = tri[~_in_polygon(c, solid)]
    a = xy[tri]
    cross = (a[:, 1, 0] - a[:, 0, 0]) * (a[:, 2, 1] - a[:, 0, 1]) - (a[:, 1, 1] - a[:, 0, 1]) * (a[:, 2, 0] - a[:, 0, 0])
    tri[cross < 0] = tri[cross < 0][:, [0, 2, 1]]
    tri = np.ascontiguousarray(tri)
    tot = 0.5 * np.abs(cross).sum()
    assert abs(tot - area) < 1e-8 * area, ("triangulation does not fill the domain", tot, area)
    # nodes no triangle uses (the solid's back corners) are dropped
    used = np.unique(tri)
    remap = -np.ones(len(xy), np.int64)
    remap[used] = np.arange(len(used))
    xy, tri = xy[used], remap[tri].astype(np.int32)
    e = np.concatenate([np.sort(np.stack([tri[:, k], tri[:, (k + 1) % 3]], 1), 1) for k in range(3)], 0)
    key = e[:, 0].astype(np.int64) * len(xy) + e[:, 1]
    _, inv, cnt = np.unique(key, return_inverse=True, return_counts=True)
    on_bnd = (cnt[inv] == 1).reshape(3, -1).T
    tags = np.full(tri.shape, -1, np.int32)
    tol = 1e-9
    for k in range(3):
        pa, pb = xy[tri[:, k]], xy[tri[:, (k + 1) % 3]]
        mid = 0.5 * (pa + pb)
        t = np.full(len(tri), 2, np.int32)  # the solid's surface unless on a side of the box
        on_box = ((np.abs(pa[:, 0]) < tol) & (np.abs(pb[:, 0]) < tol)) | \
                 ((np.abs(pa[:, 0] - W) < tol) & (np.abs(pb[:, 0] - W) < tol)) | \
                 ((np.abs(pa[:, 1]) < tol) & (np.abs(pb[:, 1]) < tol)) | \
                 ((np.abs(pa[:, 1] - H) < tol) & (np.abs(pb[:, 1] - H) < tol))
        t[on_box] = 1
        t[on_box & (np.abs(mid[:, 0]) < tol)] = 0  # x = 0: only above the solid is gas
        tags[on_bnd[:, k], k] = t[on_bnd[:, k]]
    return np.ascontiguousarray(xy), tri, tags


def diffraction_state(xy, tri, kind, gamma=1.4, m=2):
    """Cell averages of the kind's shock (Mach 5.09 at x = 1 for the step, Mach 10 at x = 3.4 for
    the wedge) moving in +x into gas at rest (rho = 1.4, p = 1), higher modes zero; and the inflow
    state (conserved, the post-shock state)."""
    spec = DIFFRACTION[kind]
    return ramp_state(xy, tri, x_shock=spec["x_shock"], mach=spec["mach"], gamma=gamma, m=m)


# ---------------------------------------------------------------------------------------------
# Initial states
# ---------------------------------------------------------------------------------------------

def sedov_1d(dx=0.01, half_width=2.0, e_total=3.2e6, e_bg=1e-12):
    """The 1D Sedov blast (Sec. 4.2.2): cells of width dx (the paper: 1/100) on
    [-(half_width + dx/2), half_width + dx/2], an odd count so that one cell is centred at 0;
    rho = 1, u = 0, E = e_bg everywhere except the centre cell, which holds E = e_total / dx.
    Returns (n, x0, x1, Q0[n][3][3]) (cell averages, higher modes zero)."""
    n = 2 * int(round(half_width / dx)) + 1
    x1 = n * dx / 2
    avg = np.zeros((n, 3))
    avg[:, 0] = 1.0
    avg[:, 2] = e_bg
    avg[n // 2, 2] = e_total / dx
    return n, -x1, x1, averages_to_modal(avg, 3)


def sedov_disk(n_target=136270, seed=0, radius=1.1, jitter=0.25):
    """Triangle mesh of the disk of the given radius (the 2D Sedov blast on an unstructured mesh,
    Sec. 4.3.2, with about n_target triangles): a jittered square lattice of spacing h inside
    radius - 0.55 h, points every about h on the circle, Delaunay.  Returns (xy, tri)."""
    g = rng(seed)
    area = math.pi * radius * radius
    h = math.sqrt(2.0 * area / n_target)
    for _ in range(6):
        m = int(math.ceil(radius / h)) + 1
        ax = np.arange(-m, m + 1) * h
        X, Y = np.meshgrid(ax, ax, indexing="xy")
        pts = np.stack([X.ravel(), Y.ravel()], 1)
        pts = pts + g.uniform(-jitter * h, jitter * h, pts.shape)
        pts = pts[np.hypot(pts[:, 0], pts[:, 1]) < radius - 0.55 * h]
        nb = int(round(2.0 * math.pi * radius / h))
        th = 2.0 * math.pi * np.arange(nb) / nb
        xy = np.concatenate([pts, radius * np.stack([np.cos(th), np.sin(th)], 1)], 0)
        n_tri = 2 * len(xy) - nb - 2  # triangles of a Delaunay triangulation with nb hull points
        if abs(n_tri - n_target) <= 0.002 * n_target:
            break
        h *= math.sqrt(n_tri / n_target)
    tri = Delaunay(xy).simplices.astype(np.int32)
    a = xy[tri]
    cross = (a[:, 1, 0] - a[:, 0, 0]) * (a[:, 2, 1] - a[:, 0, 1]) - (a[:, 1, 1] - a[:, 0, 1]) * (a[:, 2, 0] - a[:, 0, 0])
    tri[cross < 0] = tri[cross < 0][:, [0, 2, 1]]
    return xy, tri


def sedov_disk_state(xy, tri, radius=1.1, e_total=0.979264, e_bg=1e-12):
    """Initial data of the 2D Sedov blast (Sec. 4.3.2): rho = 1, u = 0, E = e_bg, and the energy
    e_total released within r_d = sqrt(pi radius^2 / n_cells) of the centre.  Reading: the
    energy is deposited on the triangles whose centroid lies within r_d, uniformly per area and
    with the exact total e_total (the quantity the blast's similarity solution depends on),
    rather than as the point function's projection.  Returns Q0[n][4][6] (cell averages, higher
    modes zero)."""
    a = np.asarray(xy)[np.asarray(tri)]
    cen = a.mean(axis=1)
    area = 0.5 * np.abs((a[:, 1, 0] - a[:, 0, 0]) * (a[:, 2, 1] - a[:, 0, 1])
                        - (a[:, 1, 1] - a[:, 0, 1]) * (a[:, 2, 0] - a[:, 0, 0]))
    r_d = math.sqrt(math.pi * radius * radius / len(tri))
    hot = np.hypot(cen[:, 0], cen[:, 1]) < r_d
    if not hot.any():
        hot[np.argmin(np.hypot(cen[:, 0], cen[:, 1]))] = True
    avg = np.zeros((len(tri), 4))
    avg[:, 0] = 1.0
    avg[:, 3] = e_bg
    avg[hot, 3] += e_total / area[hot].sum()
    return averages_to_modal(avg, 6)


def diffraction_cart(nx=390, ny=330, box=(13.0, 11.0), gamma=1.4):
    """The shock-diffraction problem over the block step (Sec. 4) on an nx x ny Cartesian mesh of
    [0, W] x [0, H] (the paper: 390 x 330, h = 1/30): the cells whose centre lies in the solid
    [0, 1] x [0, 6] are removed (their faces are reflective walls), inflow at x = 0, transparent
    elsewhere.  Returns (nx, ny, (x0, x1, y0, y1), bc, keep, Q0, inflow) with keep the nx*ny
    row-major cell flags, Q0[n_kept][4][9] the Mach 5.09 shock at x = 1 (a cell face when
    nx / W * 1 is whole) moving into gas at rest (rho = 1.4, p = 1) as cell averages (higher modes
    zero), and inflow the post-shock conserved state."""
    spec = DIFFRACTION["step"]
    W, H = box
    (sx0, sy0), (sx1, sy1) = spec["solid"][0], spec["solid"][2]
    xc = (np.arange(nx) + 0.5) * (W / nx)
    yc = (np.arange(ny) + 0.5) * (H / ny)
    X, Y = np.meshgrid(xc, yc, indexing="xy")
    solid = (X > sx0) & (X < sx1) & (Y > sy0) & (Y < sy1)
    keep = (~solid).ravel().astype(np.uint8)
    pre, post = mach_shock_states(spec["mach"], gamma=gamma)
    behind = (X < spec["x_shock"]).ravel()[keep != 0]
    prim = np.where(behind[:, None], post[None, :], pre[None, :])
    Q0 = averages_to_modal(prim_to_cons(prim, gamma), 9)
    bc = [3, 1, 1, 1]  # x-low inflow (only above the solid), x-high, y-low, y-high transparent
    return nx, ny, (0.0, W, 0.0, H), bc, keep, Q0, prim_to_cons(post[None, :], gamma)[0]


def prim_to_cons(prim, gamma):
    """(rho, u[, v], p) -> (rho, rho u[, rho v], E) along the last axis, Eq. (eos)."""
    prim = np.asarray(prim, dtype=np.float64)
    rho = prim[..., 0]
    vel = prim[..., 1:-1]
    p = prim[..., -1]
    out = np.empty_like(prim)
    out[..., 0] = rho
    out[..., 1:-1] = rho[..., None] * vel
    out[..., -1] = p / (gamma - 1.0) + 0.5 * rho * np.sum(vel * vel, axis=-1)
    return out


def tri_sample_points(xy, tri, m=4):
    """Centroids of the m^2 congruent sub-triangles of every triangle (equal-area samples)."""
    pts = []
    for a in range(m):
        for b in range(m - a):
            pts.append(((a + 1.0 / 3) / m, (b + 1.0 / 3) / m))
            if a + b < m - 1:
                pts.append(((a + 2.0 / 3) / m, (b + 2.0 / 3) / m))
    L = np.array(pts)  # barycentric (l1, l2), l0 = 1 - l1 - l2
    v = xy[tri]  # N x 3 x 2
    return v[:, 0, None, :] + L[None, :, 0, None] * (v[:, 1, None, :] - v[:, 0, None, :]) \
        + L[None, :, 1, None] * (v[:, 2, None, :] - v[:, 0, None, :])


def cart_sample_points(nx, ny, box, m=4):
    x0, x1, y0, y1 = box
    hx, hy = (x1 - x0) / nx, (y1 - y0) / ny
    s = (np.arange(m) + 0.5) / m
    ci, cj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")  # element = i + nx j
    X = x0 + (ci.ravel()[:, None, None] + s[None, :, None]) * hx
    Y = y0 + (cj.ravel()[:, None, None] + s[None, None, :]) * hy
    X, Y = np.broadcast_arrays(X, Y)
    return np.stack([X.reshape(nx * ny, -1), Y.reshape(nx * ny, -1)], axis=-1)


def averages_to_modal(avg, n_modes):
    """Piecewise-constant state: cell averages in mode 1, higher modes zero."""
    N, V = avg.shape
    Q = np.zeros((N, V, n_modes))
    Q[:, :, 0] = avg
    return Q


def cell_average_state(prim_fn, pts, gamma):
    """Cell averages of the conserved variables of a primitive-variable field, by equal-weight
    sampling at pts (N x S x dim)."""
    prim = prim_fn(pts)  # N x S x V
    return prim_to_cons(prim, gamma).mean(axis=1)


def riemann_1d_params(seed):
    """Seeded left/right primitive states: rho, p ~ U[0.1, 1], u ~ U[-1, 1]."""
    g = rng(seed)
    rl, pl, rr, pr = g.uniform(0.1, 1.0, 4)
    ul, ur = g.uniform(-1.0, 1.0, 2)
    return (rl, ul, pl), (rr, ur, pr)


def riemann_1d_state(n, seed, gamma=1.4, x0=0.0, x1=1.0, xjump=0.5):
    """Cell averages of the 1D Riemann problem on n uniform cells, jump at a cell face."""
    (rl, ul, pl), (rr, ur, pr) = riemann_1d_params(seed)
    xc = x0 + (np.arange(n) + 0.5) * (x1 - x0) / n
    prim = np.where((xc < xjump)[:, None], [rl, ul, pl], [rr, ur, pr])
    return averages_to_modal(prim_to_cons(prim, gamma), 3)


def sedov_cart_state(nx, ny, box=(-1.0, 1.0, -1.0, 1.0), gamma=1.4, e_total=0.98, p_bg=1e-10):
    """2D Sedov-type blast on an nx x ny Cartesian mesh: rho = 1, u = 0, p = p_bg background, the
    total energy e_total deposited in the 4 centre cells (mode 1 only)."""
    x0, x1, y0, y1 = box
    hx, hy = (x1 - x0) / nx, (y1 - y0) / ny
    N = nx * ny
    avg = np.zeros((N, 4))
    avg[:, 0] = 1.0
    avg[:, 3] = p_bg / (gamma - 1.0)
    ic = [nx // 2 - 1, nx // 2]
    jc = [ny // 2 - 1, ny // 2]
    for j in jc:
        for i in ic:
            avg[i + nx * j, 3] = e_total / (4.0 * hx * hy)
    return averages_to_modal(avg, 9)


def sedov_tri_state(xy, tri, r0, gamma=1.4, e_total=0.98, p_bg=1e-10):
    """Sedov-type blast on a triangle mesh: rho = 1, u = 0, p = p_bg background, the total energy
    e_total spread uniformly over the triangles whose centroid lies within r0 of the origin (cell
    averages, higher modes zero)."""
    a = np.asarray(xy)[np.asarray(tri)]
    cen = a.mean(axis=1)
    area = 0.5 * np.abs((a[:, 1, 0] - a[:, 0, 0]) * (a[:, 2, 1] - a[:, 0, 1])
                        - (a[:, 1, 1] - a[:, 0, 1]) * (a[:, 2, 0] - a[:, 0, 0]))
    hot = np.hypot(cen[:, 0], cen[:, 1]) < r0
    assert hot.any()
    avg = np.zeros((len(tri), 4))
    avg[:, 0] = 1.0
    avg[:, 3] = p_bg / (gamma - 1.0)
    avg[hot, 3] = e_total / area[hot].sum()
    return averages_to_modal(avg, 6)


def mach_shock_states(mach=10.0, rho1=1.4, p1=1.0, gamma=1.4):
    """Pre- and post-shock primitive states (rho, u, v, p) of a planar shock of Mach number `mach`
    moving in +x into gas at rest (Rankine-Hugoniot relations)."""
    c1 = math.sqrt(gamma * p1 / rho1)
    W = mach * c1
    rho2 = rho1 * (gamma + 1) * mach**2 / ((gamma - 1) * mach**2 + 2)
    p2 = p1 * (2 * gamma * mach**2 - (gamma - 1)) / (gamma + 1)
    u2 = W * (1 - rho1 / rho2)
    return np.array([rho1, 0.0, 0.0, p1]), np.array([rho2, u2, 0.0, p2])


def ramp_state(xy, tri, x_shock=0.25, mach=10.0, gamma=1.4, m=2):
    """Cell averages of a Mach `mach` shock at x = x_shock moving into the ramp channel (gas at
    rest, rho = 1.4, p = 1, ahead of it), higher modes zero; and the inflow state (conserved) for
    the x = 0 side."""
    pre, post = mach_shock_states(mach, gamma=gamma)

    def fn(pts):
        behind = pts[..., 0] < x_shock
        out = np.empty(pts.shape[:-1] + (4,))
        out[...] = pre
        out[behind] = post
        return out

    Q = averages_to_modal(cell_average_state(fn, tri_sample_points(xy, tri, m), gamma), 6)
    return Q, prim_to_cons(post[None, :], gamma)[0]


def ramp_bc(tags):
    """Boundary codes of the ramp channel's tags: inflow side -> inflow (3), outflow side and top
    -> transparent (1), floor and ramp -> reflective wall (2), interior -1."""
    tags = np.asarray(tags)
    return np.where(tags == 0, 3, np.where((tags == 1) | (tags == 3), 1, np.where(tags == 2, 2, -1))).astype(np.int32)


def four_quadrant_params(seed):
    """Seeded primitive states of the four quadrants: rho, p ~ U[0.05, 1], u, v ~ U[-1, 1]."""
    g = rng(seed)
    q = np.zeros((4, 4))
    q[:, 0] = g.uniform(0.05, 1.0, 4)
    q[:, 1] = g.uniform(-1.0, 1.0, 4)
    q[:, 2] = g.uniform(-1.0, 1.0, 4)
    q[:, 3] = g.uniform(0.05, 1.0, 4)
    return q


def four_quadrant_fn(seed, xc=0.5, yc=0.5):
    q = four_quadrant_params(seed)

    def fn(pts):
        x, y = pts[..., 0], pts[..., 1]
        quad = (x >= xc).astype(int) + 2 * (y >= yc).astype(int)
        return q[quad]

    return fn


def vortex_fn(t=0.0, eps=5.0, uinf=(1.0, 1.0), center=(0.0, 0.0), period=(10.0, 10.0), gamma=1.4):
    """Shu's isentropic vortex (strength eps) on the free stream (rho, u, v, p) = (1, uinf, 1),
    advected to time t (an exact solution of the Euler equations), nearest periodic image:
    primitive variables at points (..., 2)."""
    def fn(pts):
        xr = pts[..., 0] - center[0] - uinf[0] * t
        yr = pts[..., 1] - center[1] - uinf[1] * t
        if period is not None:
            xr = (xr + 0.5 * period[0]) % period[0] - 0.5 * period[0]
            yr = (yr + 0.5 * period[1]) % period[1] - 0.5 * period[1]
        f = np.exp(0.5 * (1.0 - xr * xr - yr * yr))
        T = 1.0 - (gamma - 1) * eps**2 / (8 * gamma * math.pi**2) * f * f
        rho = T ** (1.0 / (gamma - 1))
        return np.stack([rho, uinf[0] - eps / (2 * math.pi) * f * yr, uinf[1] + eps / (2 * math.pi) * f * xr,
                         rho * T], axis=-1)
    return fn


def vortex_shock_fn(seed, gamma=1.4, eps=5.0, box=(-5.0, 5.0, -5.0, 5.0)):
    """Isentropic vortex (strength eps) on the free stream (rho, u, v, p) = (1, 0, 0, 1),
    overlaid with a planar shock of random normal angle, position and Mach number U[1.5, 3]
    moving into the free stream; the post-shock state follows the Rankine-Hugoniot relations."""
    g = rng(seed)
    ang = g.uniform(0.0, 2.0 * math.pi)
    x0, x1, y0, y1 = box
    pos = g.uniform(0.25, 0.75)
    Ms = g.uniform(1.5, 3.0)
    nx, ny = math.cos(ang), math.sin(ang)
    # shock line through a point at fraction `pos` along the box diagonal, moving along +n
    px = x0 + pos * (x1 - x0)
    py = y0 + pos * (y1 - y0)
    # post-shock state for a shock at Mach Ms moving into (rho1, 0, p1) = (1, 0, 1)
    r1, p1 = 1.0, 1.0
    c1 = math.sqrt(gamma * p1 / r1)
    W = Ms * c1
    r2 = r1 * (gamma + 1) * Ms**2 / ((gamma - 1) * Ms**2 + 2)
    p2 = p1 * (2 * gamma * Ms**2 - (gamma - 1)) / (gamma + 1)
    u2 = W * (1 - r1 / r2)
    vx0 = 0.5 * (x0 + x1)
    vy0 = 0.5 * (y0 + y1)

    def fn(pts):
        x, y = pts[..., 0], pts[..., 1]
        r2v = (x - vx0) ** 2 + (y - vy0) ** 2
        f = np.exp(0.5 * (1.0 - r2v))
        du = -eps / (2 * math.pi) * f * (y - vy0)
        dv = eps / (2 * math.pi) * f * (x - vx0)
        T = 1.0 - (gamma - 1) * eps**2 / (8 * gamma * math.pi**2) * f * f
        rho = T ** (1.0 / (gamma - 1))
        p = rho * T
        behind = ((x - px) * nx + (y - py) * ny) < 0.0
        out = np.stack([rho, du, dv, p], axis=-1)
        post = np.array([r2, u2 * nx, u2 * ny, p2])
        out[behind] = post
        return out

    return fn


def batch_sizes(n_meshes, seed, lo=2000, hi=60000):
    """Triangle counts log-uniform in [lo, hi], mapped to lattice sizes n with 2(n-1)^2 ~ N."""
    g = rng(seed)
    N = np.exp(g.uniform(math.log(lo), math.log(hi), n_meshes))
    return [int(round(math.sqrt(x / 2.0))) + 1 for x in N]


def batch_case(n, seed, m=2, gamma=1.4, box=(-5.0, 5.0, -5.0, 5.0)):
    """One mesh of the batched workload: an n x n jittered-lattice Delaunay mesh on `box` (seed
    `seed`) with the vortex + shock field of the same seed as cell averages (m^2 samples per
    triangle), higher modes zero.  Returns (xy, tri, Q)."""
    xy, tri = lattice_delaunay(n, seed, box=box)
    Q = averages_to_modal(cell_average_state(vortex_shock_fn(seed, gamma, box=box), tri_sample_points(xy, tri, m),
                                             gamma), 6)
    return xy, tri, Q


def batch_workload(n_meshes, seed, lo=2000, hi=60000, m=2):
    """The batched workload as a generator of (xy, tri, Q): mesh b has batch_sizes(...)[b] lattice
    points per side and seed seed * 100000 + b."""
    for b, n in enumerate(batch_sizes(n_meshes, seed, lo, hi)):
        yield batch_case(n, seed * 100000 + b, m)


def _batch_case_avg(args):
    n, seed, m = args
    xy, tri, Q = batch_case(n, seed, m)
    return xy, tri, Q[:, :, 0].copy()


def batch_workload_parallel(n_meshes, seed, lo=2000, hi=60000, m=2, workers=8):
    """batch_workload as a list, built by `workers` freshly spawned processes (no state of the
    caller's process, GPU runtime included, is shared with them)."""
    import concurrent.futures
    import multiprocessing
    jobs = [(n, seed * 100000 + b, m) for b, n in enumerate(batch_sizes(n_meshes, seed, lo, hi))]
    ctx = multiprocessing.get_context("spawn")
    with concurrent.futures.ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        out = list(ex.map(_batch_case_avg, jobs, chunksize=4))
    return [(xy, tri, averages_to_modal(avg, 6)) for xy, tri, avg in out]


def mlp_init(seed, n_in=48, n_h=64):
    """Initial parameters of the indicator network (flat float32, layout W1, b1, W2, b2, w3, b3):
    weights uniform in +-sqrt(6 / fan_in), biases uniform in +-0.05, seeded."""
    g = rng(seed)
    parts = [g.uniform(-1, 1, n_in * n_h) * math.sqrt(6.0 / n_in), g.uniform(-0.05, 0.05, n_h),
             g.uniform(-1, 1, n_h * n_h) * math.sqrt(6.0 / n_h), g.uniform(-0.05, 0.05, n_h),
             g.uniform(-1, 1, n_h) * math.sqrt(6.0 / n_h), g.uniform(-0.05, 0.05, 1)]
    return np.concatenate(parts).astype(np.float32)


def random_modal_state(N, dim, n_modes, seed, amp=0.3, gamma=1.4, p_range=(0.3, 1.5), rough_frac=0.0,
                       rough_amp=2.0):
    """Random modal coefficients for parity tests: cell averages from random positive primitive
    states, higher modes uniform in [-amp, amp] times the average's scale; a fraction rough_frac
    of the cells get rough_amp instead, which drives point densities and pressures negative and
    so exercises the limiters."""
    g = rng(seed)
    V = dim + 2
    prim = np.zeros((N, V))
    prim[:, 0] = g.uniform(0.3, 1.5, N)
    prim[:, 1:1 + dim] = g.uniform(-1.0, 1.0, (N, dim))
    prim[:, -1] = g.uniform(p_range[0], p_range[1], N)
    avg = prim_to_cons(prim, gamma)
    Q = np.zeros((N, V, n_modes))
    Q[:, :, 0] = avg
    scale = np.abs(avg) + 0.2
    a = np.full(N, amp)
    if rough_frac > 0:
        a[g.uniform(0, 1, N) < rough_frac] = rough_amp
    Q[:, :, 1:] = g.uniform(-1.0, 1.0, (N, V, n_modes - 1)) * (a[:, None] * scale)[:, :, None] / np.sqrt(n_modes)
    return Q


def bowl_prim_tet(xyz, tet, pts, seed, rho_range=(1e-6, 1.0), p_range=(1e-8, 1.0), depth=0.02, curv=6.0, spread=3.0):
    """The same adversarial fields on tetrahedra: in every tetrahedron a bowl-shaped density and
    pressure (low at the centroid) of random log-uniform scale, and a random velocity plus an
    outward spread from the centroid (h = the cube root of 6 |T|).  pts[N][P][3] are sample points
    of each tetrahedron; returns prim[N][P][5]."""
    g = rng(seed)
    N = len(tet)
    v = xyz[tet]
    c = v.mean(axis=1)
    vol = np.abs(np.einsum("ij,ij->i", v[:, 1] - v[:, 0], np.cross(v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]))) / 6.0
    h = np.cbrt(6.0 * vol)
    rs = np.exp(g.uniform(math.log(rho_range[0]), math.log(rho_range[1]), N))
    ps = np.exp(g.uniform(math.log(p_range[0]), math.log(p_range[1]), N))
    vel = g.uniform(-2.0, 2.0, (N, 3))
    d = (pts - c[:, None, :]) / h[:, None, None]
    r2 = np.sum(d * d, axis=-1)
    rho = rs[:, None] * (depth + curv * r2)
    p = ps[:, None] * (depth + curv * r2)
    u = [vel[:, None, a] + spread * d[..., a] for a in range(3)]
    return np.stack([rho, u[0], u[1], u[2], p], axis=-1)


def bowl_prim(xy, tri, pts, seed, rho_range=(1e-6, 1.0), p_range=(1e-8, 1.0), depth=0.02, curv=6.0, spread=3.0):
    """Adversarial per-cell primitive fields for exercising the flux limiter: in every triangle a
    bowl-shaped density and pressure (low at the centroid, high at the edges) of random
    log-uniform scale, and a random velocity plus an outward spread from the centroid.
    pts[N][P][2] are sample points of each triangle; returns prim[N][P][4]."""
    g = rng(seed)
    N = len(tri)
    c = xy[tri].mean(axis=1)
    v = xy[tri]
    area = 0.5 * np.abs((v[:, 1, 0] - v[:, 0, 0]) * (v[:, 2, 1] - v[:, 0, 1]) - (v[:, 1, 1] - v[:, 0, 1]) * (v[:, 2, 0] - v[:, 0, 0]))
    h = np.sqrt(2.0 * area)
    rs = np.exp(g.uniform(math.log(rho_range[0]), math.log(rho_range[1]), N))
    ps = np.exp(g.uniform(math.log(p_range[0]), math.log(p_range[1]), N))
    vel = g.uniform(-2.0, 2.0, (N, 2))
    d = (pts - c[:, None, :]) / h[:, None, None]
    r2 = np.sum(d * d, axis=-1)
    rho = rs[:, None] * (depth + curv * r2)
    p = ps[:, None] * (depth + curv * r2)
    u = vel[:, None, 0] + spread * d[..., 0]
    w = vel[:, None, 1] + spread * d[..., 1]
    return np.stack([rho, u, w, p], axis=-1)
