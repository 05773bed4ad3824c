"""TEST INFRASTRUCTURE ONLY -- Python access to the FP64 CPU oracle (lxw_oracle.cpp).

The oracle is a plain, slow implementation of the positivity-preserving Lax-Wendroff DG step
(Moe, Rossmanith, Seal, arXiv:1601.08145) that the GPU library is checked against.  Only the
test-suite, the smoke entry point and the CPU-baseline leg of the benchmark use it; the GPU
library never imports, links or calls anything here.

Array layouts follow the library's public interface: modal coefficients Q[n_elem][n_var][n_modes]
(row-major, float64), per-(element, local edge) quantities [n_elem][n_edges_per_elem](...).
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lxw_oracle.cpp")
LIB = os.path.join(HERE, "liblxw_oracle.so")

LINE, QUAD, TRI, TET = 0, 1, 2, 3
BC_PERIODIC, BC_TRANSPARENT, BC_REFLECTIVE, BC_INFLOW = 0, 1, 2, 3

STAGE_QLIM, STAGE_THETA_MOM, STAGE_VOL, STAGE_FLXW, STAGE_FLXF = 0, 1, 2, 3, 4
STAGE_LAM_IK, STAGE_C_IK, STAGE_LAM_E, STAGE_QUPD, STAGE_THETA_SC, STAGE_SDT = 5, 6, 7, 8, 9, 10
STAGE_QDERIV = 11


def build():
    """Compile the oracle: C++17, FP64, no fast-math, no FMA contraction, OpenMP."""
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", SRC, "-o", LIB + ".tmp"]
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i, d = ctypes.c_int, ctypes.c_double
        sig = {
            "ora_mesh_1d": (P, [i, d, d, i, i]),
            "ora_num_threads": (i, []),
            "ora_set_num_threads": (None, [i]),
            "ora_mesh_cart": (P, [i, i, d, d, d, d, ip, u8p, i]),
            "ora_mesh_tri": (P, [i, dp, i, ip, ip, dp]),
            "ora_mesh_tet": (P, [i, dp, i, ip, ip, dp]),
            "ora_mesh_edges": (None, [P, ip, ip, ip, ip, dp]),
            "ora_mesh_point_order": (None, [P, ip]),
            "ora_last_error": (ctypes.c_char_p, []),
            "ora_mesh_free": (None, [P]),
            "ora_mesh_info": (None, [P, ip]),
            "ora_mesh_geom": (None, [P, dp, dp, ip, ip]),
            "ora_solver_new": (P, [P, d, d, d, d, i, dp]),
            "ora_solver_free": (None, [P]),
            "ora_force_theta": (None, [P, d]),
            "ora_set_exact_theta": (None, [P, i]),
            "ora_set_s_avg": (None, [P, i]),
            "ora_set_shock_mask": (None, [P, P]),
            "ora_set_state": (None, [P, dp, d]),
            "ora_get_state": (None, [P, dp, dp]),
            "ora_step": (i, [P, d, dp]),
            "ora_error_elem": (i, [P]),
            "ora_error_msg": (ctypes.c_char_p, [P]),
            "ora_stage": (i, [P, i, dp]),
            "ora_ref_info": (None, [i, i, ip]),
            "ora_ref_tables": (None, [i, i, dp, dp, dp, dp, dp]),
            "ora_phi": (d, [i, i, i, dp, i, i, i]),
            "ora_mesh_set_degree": (i, [P, i]),
            "ora_flux_3vp": (None, [i, d, dp, i, dp, dp, dp, dp]),
            "ora_ft4": (None, [i, d, d, dp, dp, dp, dp, dp]),
            "ora_flux": (None, [i, d, dp, i, dp]),
            "ora_flux_jvp": (None, [i, d, dp, i, dp, dp]),
            "ora_flux_hvp": (None, [i, d, dp, i, dp, dp, dp]),
            "ora_ft": (None, [i, d, d, dp, dp, dp, dp]),
            "ora_mu_solve": (d, [i, d, d, dp, dp]),
            "ora_moment_limit": (d, [P, dp]),
            "ora_shock_limit": (d, [P, dp, i, dp]),
            "ora_quad_points": (None, [P, dp]),
            "ora_project": (None, [P, dp, dp]),
            "ora_eval": (None, [P, i, dp, dp, dp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class RefElem:
    """Reference element tables of kind LINE, QUAD, TRI or TET and polynomial degree 2 (or 3:
    LINE, TRI)."""

    def __init__(self, kind, degree=2):
        L = lib()
        info = np.zeros(5, np.int32)
        L.ora_ref_info(kind, degree, _i(info))
        self.kind = kind
        self.degree = degree
        self.dim, self.ML, self.K, self.NI, self.NQE = (int(x) for x in info)
        self.C = np.zeros((self.ML, self.ML))
        self.xi_int = np.zeros((self.NI, self.dim))
        self.w_int = np.zeros(self.NI)
        self.xi_edge = np.zeros((self.K, self.NQE, self.dim))
        self.om_edge = np.zeros(self.NQE)
        L.ora_ref_tables(kind, degree, _d(self.C), _d(self.xi_int), _d(self.w_int), _d(self.xi_edge),
                         _d(self.om_edge))

    def phi(self, l, xi, da=0, db=0, dc=0):
        xi = f64(np.atleast_1d(xi))
        return lib().ora_phi(self.kind, self.degree, l, _d(xi), da, db, dc)


class Mesh:
    def __init__(self, handle, degree=2):
        if not handle:
            raise ValueError("oracle mesh construction failed: " + lib().ora_last_error().decode())
        self.h = handle
        if degree != 2 and lib().ora_mesh_set_degree(self.h, degree) != 0:
            raise ValueError(f"no degree-{degree} elements of this kind")
        self.degree = degree
        info = np.zeros(8, np.int32)
        lib().ora_mesh_info(self.h, _i(info))
        self.kind, self.dim, self.N, self.E, self.ML, self.K, self.NI, self.NQE = (int(x) for x in info)
        self.V = self.dim + 2
        self.area = np.zeros(self.N)
        self.perim = np.zeros(self.N)
        self.nbr = np.zeros((self.N, self.K), np.int32)
        self.nbr_k = np.zeros((self.N, self.K), np.int32)
        lib().ora_mesh_geom(self.h, _d(self.area), _d(self.perim), _i(self.nbr), _i(self.nbr_k))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ora_mesh_free(self.h)
            self.h = None

    @staticmethod
    def line(n, x0, x1, bc_left, bc_right, degree=2):
        return Mesh(lib().ora_mesh_1d(n, x0, x1, bc_left, bc_right), degree)

    @staticmethod
    def cart(nx, ny, x0, x1, y0, y1, bc, keep=None, wall_bc=2):
        """Cartesian Q2 mesh; keep (nx*ny flags, cell (i, j) at i + nx*j) removes cells, whose
        faces become boundaries of type wall_bc (reflective by default)."""
        b = i32(bc)
        k = None
        if keep is not None:
            k = np.ascontiguousarray(np.asarray(keep, dtype=np.uint8).reshape(-1))
            if k.size != nx * ny:
                raise ValueError("keep needs nx * ny flags")
        return Mesh(lib().ora_mesh_cart(nx, ny, x0, x1, y0, y1, _i(b),
                                        k.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)) if k is not None else None,
                                        int(wall_bc)))

    @staticmethod
    def tri(xy, tri, bnd=None, period=None, degree=2):
        xy = f64(xy)
        tri = i32(tri)
        b = i32(bnd) if bnd is not None else None
        p = f64(period) if period is not None else None
        h = lib().ora_mesh_tri(len(xy), _d(xy), len(tri), _i(tri), _i(b) if b is not None else None,
                               _d(p) if p is not None else None)
        return Mesh(h, degree)

    @staticmethod
    def tet(xyz, tet, bnd=None, period=None):
        """Tetrahedral P2 mesh: nodes xyz (n x 3), tetrahedra (n_tet x 4, positively oriented),
        boundary codes per (tetrahedron, face k opposite vertex k), period (3 lengths)."""
        xyz = f64(xyz)
        tet = i32(tet)
        b = i32(bnd) if bnd is not None else None
        p = f64(period) if period is not None else None
        h = lib().ora_mesh_tet(len(xyz), _d(xyz), len(tet), _i(tet), _i(b) if b is not None else None,
                               _d(p) if p is not None else None)
        return Mesh(h)

    def edges(self):
        """(e_i, e_ki, e_j, e_kj, n_e[E][3]) of the edges (faces in 3D)."""
        ei, ki, ej, kj = (np.zeros(self.E, np.int32) for _ in range(4))
        n = np.zeros((self.E, 3))
        lib().ora_mesh_edges(self.h, _i(ei), _i(ki), _i(ej), _i(kj), _d(n))
        return ei, ki, ej, kj, n

    def point_order(self):
        """fmap[N][K][NQE]: local edge point jl of (i, k) is point fmap of the edge in i_e's order."""
        f = np.zeros((self.N, self.K, self.NQE), np.int32)
        lib().ora_mesh_point_order(self.h, _i(f))
        return f

    def quad_points(self):
        x = np.zeros((self.N, self.NI, self.dim))
        lib().ora_quad_points(self.h, _d(x))
        return x

    def project(self, vals):
        """L2 projection of point values at the interior quadrature points (N x NI x V)."""
        vals = f64(vals)
        Q = np.zeros((self.N, self.V, self.ML))
        lib().ora_project(self.h, _d(vals), _d(Q))
        return Q


class OracleError(RuntimeError):
    def __init__(self, code, elem, msg):
        super().__init__(f"oracle status {code}: {msg}")
        self.code, self.elem = code, elem


class Solver:
    def __init__(self, mesh, gamma=1.4, cfl=0.08, eps0=1e-12, alpha0=500.0, shock=True, inflow=None,
                 exact_theta=False, s_from_averages=False):
        self.mesh = mesh
        inf = f64(inflow) if inflow is not None else None
        self.h = lib().ora_solver_new(mesh.h, gamma, cfl, eps0, alpha0, int(bool(shock)),
                                      _d(inf) if inf is not None else None)
        if exact_theta:
            lib().ora_set_exact_theta(self.h, 1)
        if s_from_averages:
            lib().ora_set_s_avg(self.h, 1)
        self.gamma = gamma

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ora_solver_free(self.h)
            self.h = None

    def set_shock_mask(self, mask):
        """Cells on which the shock-capturing limiter may act (None: all), for the learned form."""
        if mask is None:
            lib().ora_set_shock_mask(self.h, None)
            return
        m = np.ascontiguousarray(np.asarray(mask) != 0, dtype=np.uint8)
        assert m.shape == (self.mesh.N,)
        self._mask = m
        lib().ora_set_shock_mask(self.h, m.ctypes.data_as(ctypes.c_void_p))

    def force_theta(self, th):
        """Test hook: replace every edge blending factor Lambda_e by th (th < 0 switches it off)."""
        lib().ora_force_theta(self.h, th)

    def set_state(self, Q, t=0.0):
        Q = f64(Q)
        assert Q.shape == (self.mesh.N, self.mesh.V, self.mesh.ML)
        lib().ora_set_state(self.h, _d(Q), t)

    def get_state(self):
        Q = np.zeros((self.mesh.N, self.mesh.V, self.mesh.ML))
        t = np.zeros(1)
        lib().ora_get_state(self.h, _d(Q), _d(t))
        return Q, float(t[0])

    def step(self, T=np.inf, check=True):
        dt = np.zeros(1)
        st = lib().ora_step(self.h, T, _d(dt))
        if st != 0 and check:
            raise OracleError(st, lib().ora_error_elem(self.h), lib().ora_error_msg(self.h).decode())
        return st, float(dt[0])

    def advance(self, T, max_steps=10**9):
        n = 0
        while self.get_state()[1] < T and n < max_steps:
            self.step(T)
            n += 1
        return n

    def stage(self, stage):
        m = self.mesh
        shapes = {
            STAGE_QLIM: (m.N, m.V, m.ML), STAGE_THETA_MOM: (m.N,), STAGE_VOL: (m.N, m.V, m.ML),
            STAGE_FLXW: (m.N, m.K, m.V), STAGE_FLXF: (m.N, m.K, m.V), STAGE_LAM_IK: (m.N, m.K),
            STAGE_C_IK: (m.N, m.K), STAGE_LAM_E: (m.N, m.K), STAGE_QUPD: (m.N, m.V, m.ML),
            STAGE_THETA_SC: (m.N,), STAGE_SDT: (2,), STAGE_QDERIV: (m.N, m.NI, 3, m.V),
        }
        out = np.zeros(shapes[stage])
        if lib().ora_stage(self.h, stage, _d(out)) != 0:
            raise ValueError(stage)
        return out

    def moment_limit(self, Qi):
        Qi = f64(Qi).copy()
        th = lib().ora_moment_limit(self.h, _d(Qi))
        return th, Qi

    def shock_limit(self, Qall, i, Qi=None):
        """The shock-capturing limiter on element i: its coefficients Qi (default Qall[i]), the
        neighbours' averages from Qall.  Returns (theta, limited coefficients)."""
        Qall = f64(Qall)
        assert Qall.shape == (self.mesh.N, self.mesh.V, self.mesh.ML)
        Qi = f64(Qall[i] if Qi is None else Qi).copy()
        th = lib().ora_shock_limit(self.h, _d(Qall), int(i), _d(Qi))
        return th, Qi

    def eval_points(self, xi):
        """q^h at reference points xi (P x dim) of every element -> (N x P x V), coords (N x P x dim)."""
        xi = f64(np.atleast_2d(xi))
        P = xi.shape[0]
        out = np.zeros((self.mesh.N, P, self.mesh.V))
        x = np.zeros((self.mesh.N, P, self.mesh.dim))
        lib().ora_eval(self.h, P, _d(xi), _d(out), _d(x))
        return out, x


def num_threads():
    return int(lib().ora_num_threads())


def set_num_threads(n):
    """OpenMP threads of the oracle's loops (results do not depend on it)."""
    lib().ora_set_num_threads(int(n))


def flux(q, d=0, gamma=1.4):
    q = f64(q)
    dim = len(q) - 2
    F = np.zeros(len(q))
    lib().ora_flux(dim, gamma, _d(q), d, _d(F))
    return F


def flux_jvp(q, x, d=0, gamma=1.4):
    q, x = f64(q), f64(x)
    out = np.zeros(len(q))
    lib().ora_flux_jvp(len(q) - 2, gamma, _d(q), d, _d(x), _d(out))
    return out


def flux_hvp(q, x, y, d=0, gamma=1.4):
    q, x, y = f64(q), f64(x), f64(y)
    out = np.zeros(len(q))
    lib().ora_flux_hvp(len(q) - 2, gamma, _d(q), d, _d(x), _d(y), _d(out))
    return out


def ft(q, qt, qtt, dt, gamma=1.4):
    q, qt, qtt = f64(q), f64(qt), f64(qtt)
    dim = len(q) - 2
    out = np.zeros((dim, len(q)))
    lib().ora_ft(dim, gamma, dt, _d(q), _d(qt), _d(qtt), _d(out))
    return out


def flux_3vp(q, x, y, z, d=0, gamma=1.4):
    q, x, y, z = f64(q), f64(x), f64(y), f64(z)
    out = np.zeros(len(q))
    lib().ora_flux_3vp(len(q) - 2, gamma, _d(q), d, _d(x), _d(y), _d(z), _d(out))
    return out


def ft4(q, qt, qtt, qttt, dt, gamma=1.4):
    q, qt, qtt, qttt = f64(q), f64(qt), f64(qtt), f64(qttt)
    dim = len(q) - 2
    out = np.zeros((dim, len(q)))
    lib().ora_ft4(dim, gamma, dt, _d(q), _d(qt), _d(qtt), _d(qttt), _d(out))
    return out


def mu_solve(qL, qa, eps_p, gamma=1.4):
    qL, qa = f64(qL), f64(qa)
    return lib().ora_mu_solve(len(qL) - 2, gamma, eps_p, _d(qL), _d(qa))
