"""Shared test helpers: independent mesh geometry, exact solutions, error norms.

Nothing here is imported by the GPU library or by the oracle."""
import math

import numpy as np

G = 1.4


def pressure(q, gamma=G):
    q = np.asarray(q)
    dim = q.shape[-1] - 2
    kin = 0.5 * np.sum(q[..., 1:1 + dim] ** 2, axis=-1) / q[..., 0]
    return (gamma - 1) * (q[..., -1] - kin)


def euler_flux_n(q, n, gamma=G):
    """n . F(q) for states q (..., V) and normals n (..., dim): Sec. 1.5 flux, written directly."""
    q = np.asarray(q)
    dim = q.shape[-1] - 2
    rho = q[..., 0]
    mom = q[..., 1:1 + dim]
    E = q[..., -1]
    p = pressure(q, gamma)
    un = np.sum(mom * n, axis=-1) / rho
    out = np.empty_like(q)
    out[..., 0] = rho * un
    out[..., 1:1 + dim] = mom * un[..., None] + p[..., None] * n
    out[..., -1] = un * (E + p)
    return out


def tri_geometry(xy, tri):
    """Outward normals n[t][k] (length = edge length) of edge k = (v_k, v_k+1), areas, and
    neighbours (t', k') found by matching vertex pairs (-1 on the boundary)."""
    v = xy[tri]
    nrm = np.zeros((len(tri), 3, 2))
    for k in range(3):
        d = v[:, (k + 1) % 3] - v[:, k]
        nrm[:, k, 0] = d[:, 1]
        nrm[:, k, 1] = -d[:, 0]
    area = 0.5 * ((v[:, 1, 0] - v[:, 0, 0]) * (v[:, 2, 1] - v[:, 0, 1]) - (v[:, 1, 1] - v[:, 0, 1]) * (v[:, 2, 0] - v[:, 0, 0]))
    key = {}
    nb = -np.ones((len(tri), 3), np.int64)
    for t in range(len(tri)):
        for k in range(3):
            a, b = tri[t, k], tri[t, (k + 1) % 3]
            kk = (min(a, b), max(a, b))
            if kk in key:
                t2, k2 = key.pop(kk)
                nb[t, k] = t2
                nb[t2, k2] = t
            else:
                key[kk] = (t, k)
    return nrm, area, nb


def vortex_prim(x, y, t, eps=5.0, uinf=(1.0, 1.0), center=(0.0, 0.0), gamma=G, period=None):
    """Shu's isentropic vortex advected with uinf; with a period the nearest image is used."""
    xr = x - center[0] - uinf[0] * t
    yr = y - center[1] - uinf[1] * t
    if period is not None:
        xr = (xr + 0.5 * period[0]) % period[0] - 0.5 * period[0]
        yr = (yr + 0.5 * period[1]) % period[1] - 0.5 * period[1]
    r2 = xr * xr + yr * yr
    f = np.exp(0.5 * (1 - r2))
    T = 1 - (gamma - 1) * eps**2 / (8 * gamma * math.pi**2) * f * f
    rho = T ** (1 / (gamma - 1))
    return np.stack([rho, uinf[0] - eps / (2 * math.pi) * f * yr, uinf[1] + eps / (2 * math.pi) * f * xr, rho * T], -1)


def e3_prim(x, y, t):
    """The paper's smooth near-vacuum advection (Sec. 4.3.1, Eq. (exactsolnconv))."""
    rho = 1 - 0.9999 * np.sin(2 * np.pi * (x - t)) * np.sin(2 * np.pi * y)
    one = np.ones_like(rho)
    return np.stack([rho, one, 0 * one, one], -1)


def cons(prim, gamma=G):
    prim = np.asarray(prim)
    dim = prim.shape[-1] - 2
    out = np.empty_like(prim)
    out[..., 0] = prim[..., 0]
    out[..., 1:1 + dim] = prim[..., :1] * prim[..., 1:1 + dim]
    out[..., -1] = prim[..., -1] / (gamma - 1) + 0.5 * prim[..., 0] * np.sum(prim[..., 1:1 + dim] ** 2, axis=-1)
    return out


def error_rule(kind, n=6):
    """An independent Gauss rule on the reference element (points, weights summing to 1), of
    higher degree than the method's own rules: kind 0 line [-1,1], 1 square [-1,1]^2,
    2 triangle (0,0),(1,0),(0,1) by the collapsed (Duffy) map."""
    x, w = np.polynomial.legendre.leggauss(n)
    if kind == 0:
        return x[:, None], w / 2.0
    if kind == 1:
        X, Y = np.meshgrid(x, x, indexing="ij")
        return np.stack([X.ravel(), Y.ravel()], 1), np.outer(w, w).ravel() / 4.0
    u = 0.5 * (x + 1)
    wu = 0.5 * w
    U, V = np.meshgrid(u, u, indexing="ij")
    W = np.outer(wu, wu) * (1 - U)
    return np.stack([U.ravel(), ((1 - U) * V).ravel()], 1), 2.0 * W.ravel()


def error_rule_tet(n=5):
    """An independent collapsed Gauss rule on the reference tetrahedron (0,0,0),(1,0,0),(0,1,0),
    (0,0,1) (points, weights summing to 1), exact to degree 2n - 1."""
    from scipy.special import roots_jacobi
    x0, w0 = roots_jacobi(n, 0, 0)
    x1, w1 = roots_jacobi(n, 1, 0)
    x2, w2 = roots_jacobi(n, 2, 0)
    U, Vv, W = np.meshgrid(0.5 * (1 + x0), 0.5 * (1 + x1), 0.5 * (1 + x2), indexing="ij")
    wt = (6 / 64) * w0[:, None, None] * w1[None, :, None] * w2[None, None, :]
    pts = np.stack([U * (1 - Vv) * (1 - W), Vv * (1 - W), W], -1).reshape(-1, 3)
    return pts, wt.ravel()


def l2_error(solver, ref, exact_fn, var=0):
    """L2 error of variable `var` of q^h against exact_fn (x -> conserved), measured with an
    independent higher-order rule (the method's own rule can coincide with interpolation
    points of the projection and hide the error)."""
    m = solver.mesh
    pts, w = error_rule(ref.kind)
    qh, x = solver.eval_points(pts)
    ex = exact_fn(x)
    err2 = np.sum((qh[..., var] - ex[..., var]) ** 2 * w[None, :], axis=1) * m.area
    return math.sqrt(err2.sum() / m.area.sum())


def rel_l1(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.sum(np.abs(b))
    return float(np.sum(np.abs(a - b)) / (den if den > 0 else 1.0))
