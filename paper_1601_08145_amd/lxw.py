"""Python binding of the LxW-DG library (include/lxw.h): argument marshalling only.

Every step of the method runs in the library's HIP kernels; this module converts arrays, passes
pointers and sizes, and turns status codes into exceptions.  PyTorch is used for device memory and
streams (a solver runs on a torch stream; states may be torch tensors on the GPU).  torch is
imported before the library is loaded so that both use the same HIP runtime.

There is no fallback: if liblxw.so is missing, importing this module raises.
"""
import ctypes
import os

import numpy as np
import torch  # noqa: F401  (must precede loading liblxw.so: one HIP runtime per process)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblxw.so")

LXW_OK = 0
ERRORS = {-1: "LXW_ERR_ARG", -2: "LXW_ERR_UNSUPPORTED", -3: "LXW_ERR_MESH", -4: "LXW_ERR_STATE",
          -5: "LXW_ERR_POSITIVITY", -6: "LXW_ERR_NONFINITE", -7: "LXW_ERR_CFL", -8: "LXW_ERR_DEVICE",
          -9: "LXW_ERR_OOM"}
BC_PERIODIC, BC_TRANSPARENT, BC_REFLECTIVE, BC_INFLOW = 0, 1, 2, 3
SPEED_POINTS, SPEED_AVERAGES = 0, 1
LINE, QUAD, TRI, TET = 0, 1, 2, 3
FP64, FP32_MIXED = 0, 1
SHOCK_OFF, SHOCK_PLAIN = 0, 1
HOST_PTR, DEVICE_PTR, STATE_UNCHECKED = 0, 1, 2
STAGE_QLIM, STAGE_THETA, STAGE_VOL, STAGE_FLXW, STAGE_FLXF = 0, 1, 2, 3, 4
STAGE_C, STAGE_LAME, STAGE_QUPD, STAGE_THETA_SC, STAGE_SDT = 6, 7, 8, 9, 10
K_PRE, K_DT, K_ELEM, K_EDGE, K_FLIM, K_UPDATE, K_FINAL, K_IND, K_COUNT = 0, 1, 2, 3, 4, 5, 6, 7, 8
KERNEL_NAMES = ["k_pre", "k_dt", "k_elem", "k_edge", "k_flim", "k_update", "k_final", "k_ind"]


class LxwError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))
        self.msg = msg


class Params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("degree", ctypes.c_int32), ("cfl", ctypes.c_double),
                ("eps0", ctypes.c_double), ("alpha0", ctypes.c_double), ("precision", ctypes.c_int32),
                ("shock", ctypes.c_int32), ("inflow", ctypes.c_double * 4), ("theta_exact", ctypes.c_int32),
                ("wave_speed", ctypes.c_int32)]


class MeshInfo(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dim", ctypes.c_int32), ("n_elem", ctypes.c_int32),
                ("n_edge", ctypes.c_int32), ("n_var", ctypes.c_int32), ("n_modes", ctypes.c_int32),
                ("n_faces", ctypes.c_int32), ("min_area", ctypes.c_double), ("max_area", ctypes.c_double)]


class Tune(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32 * 8), ("persistent", ctypes.c_int32)]


class Adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_double), ("w_pos", ctypes.c_double), ("w_neg", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("t", ctypes.c_double), ("last_dt", ctypes.c_double),
                ("last_s", ctypes.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    sig = {
        "lxw_params_default": [ctypes.POINTER(Params)],
        "lxw_mesh_create_1d": [I32, D, D, I32, I32, ctypes.POINTER(P)],
        "lxw_mesh_create_cart": [I32, I32, D, D, D, D, ip, ctypes.POINTER(P)],
        "lxw_mesh_create_cart_masked": [I32, I32, D, D, D, D, ip, ctypes.POINTER(ctypes.c_uint8), I32,
                                        ctypes.POINTER(P)],
        "lxw_mesh_create_tri": [I32, dp, I32, ip, ip, dp, ctypes.POINTER(P)],
        "lxw_mesh_create_tet": [I32, dp, I32, ip, ip, dp, ctypes.POINTER(P)],
        "lxw_mesh_destroy": [P],
        "lxw_mesh_get_info": [P, ctypes.POINTER(MeshInfo)],
        "lxw_refelem_info": [I32, ip, dp, dp, dp],
        "lxw_refelem_info_deg": [I32, I32, ip, dp, dp, dp],
        "lxw_solver_create": [P, ctypes.POINTER(Params), P, ctypes.POINTER(P)],
        "lxw_solver_destroy": [P],
        "lxw_set_state": [P, P, D, I32],
        "lxw_get_state": [P, P, dp, I32],
        "lxw_step": [P, D, dp],
        "lxw_advance": [P, D, I64, ctypes.POINTER(Stats)],
        "lxw_run_steps": [P, I64],
        "lxw_sync": [P],
        "lxw_set_debug": [P, I32],
        "lxw_debug_stage": [P, I32, dp],
        "lxw_set_timing": [P, I32],
        "lxw_kernel_times": [P, dp, ctypes.POINTER(ctypes.c_int64)],
        "lxw_set_graph": [P, I32],
        "lxw_get_tune": [P, ctypes.POINTER(Tune)],
        "lxw_set_tune": [P, ctypes.POINTER(Tune)],
        "lxw_autotune": [P, I32, ctypes.POINTER(Tune)],
        "lxw_batch_create": [I32, ctypes.POINTER(P), ctypes.POINTER(Params), P, ctypes.POINTER(P)],
        "lxw_batch_destroy": [P],
        "lxw_batch_set_state": [P, I32, P, D, I32],
        "lxw_batch_get_state": [P, I32, P, dp, I32],
        "lxw_batch_advance_steps": [P, I64],
        "lxw_batch_stats": [P, I32, ctypes.POINTER(Stats)],
        "lxw_indicator_create": [P, P, ctypes.POINTER(P)],
        "lxw_indicator_destroy": [P],
        "lxw_indicator_get_params": [P, P],
        "lxw_indicator_set_params": [P, P],
        "lxw_indicator_save": [P, ctypes.c_char_p],
        "lxw_indicator_load": [P, ctypes.c_char_p],
        "lxw_indicator_predict": [P, P, I32, P],
        "lxw_indicator_grad": [P, P, P, I32, D, D, P, dp],
        "lxw_indicator_grad_noalloc": [P, P, P, I32, D, D, P, P],
        "lxw_indicator_train": [P, P, P, I32, P, I32, I32, ctypes.POINTER(Adam), dp],
        "lxw_indicator_collect": [P, P, P, I32],
        "lxw_solver_set_indicator": [P, P, D, D],
        "lxw_indicator_decisions": [P, P, P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int32
    L.lxw_last_error.argtypes = []
    L.lxw_last_error.restype = ctypes.c_char_p
    L.lxw_batch_solver.argtypes = [P]
    L.lxw_batch_solver.restype = P
    return L


_L = _load()


def lib():
    return _L


def _check(code):
    if code != LXW_OK:
        raise LxwError(code, _L.lxw_last_error().decode())


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def default_params(**kw):
    p = Params()
    _check(_L.lxw_params_default(ctypes.byref(p)))
    for k, v in kw.items():
        if k == "inflow":
            for c in range(4):
                p.inflow[c] = float(v[c])
        elif k in dict(Params._fields_):
            setattr(p, k, v)
        else:
            raise TypeError(f"unknown solver parameter {k!r}")
    return p


def n_modes(kind, degree=2):
    return {(LINE, 2): 3, (QUAD, 2): 9, (TRI, 2): 6, (TET, 2): 10, (LINE, 3): 4, (TRI, 3): 10}[(kind, degree)]


def refelem_info(kind, degree=2):
    """Interior quadrature points xi[n][dim], weights w[n] (sum 1) and basis values phi[n][n_modes]
    at polynomial degree 2 (or 3 on lines and triangles)."""
    n = ctypes.c_int32(0)
    _check(_L.lxw_refelem_info_deg(kind, degree, ctypes.byref(n), None, None, None))
    dim = 1 if kind == LINE else (3 if kind == TET else 2)
    xi = np.zeros((n.value, dim))
    w = np.zeros(n.value)
    phi = np.zeros((n.value, n_modes(kind, degree)))
    _check(_L.lxw_refelem_info_deg(kind, degree, ctypes.byref(n), _dp(xi), _dp(w), _dp(phi)))
    return xi, w, phi


class Mesh:
    def __init__(self, handle, kind, verts):
        self.h = handle
        self.kind = kind
        info = MeshInfo()
        _check(_L.lxw_mesh_get_info(self.h, ctypes.byref(info)))
        self.info = info
        self.N, self.E = info.n_elem, info.n_edge
        self.V, self.ML, self.K, self.dim = info.n_var, info.n_modes, info.n_faces, info.dim
        self.verts = verts  # caller-order element vertex coordinates (N x nv x dim), for projection

    def __del__(self, _destroy=_L.lxw_mesh_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    @staticmethod
    def line(n, x0, x1, bc_left, bc_right):
        h = ctypes.c_void_p()
        _check(_L.lxw_mesh_create_1d(n, x0, x1, bc_left, bc_right, ctypes.byref(h)))
        xs = np.linspace(x0, x1, n + 1)
        return Mesh(h, LINE, np.stack([xs[:-1], xs[1:]], 1)[:, :, None])

    @staticmethod
    def cart(nx, ny, x0, x1, y0, y1, bc, keep=None, wall_bc=BC_REFLECTIVE):
        """Cartesian Q2 mesh; keep (nx*ny flags, cell (i, j) at i + nx*j) removes the cells whose flag
        is 0, their faces becoming boundaries of type wall_bc; the kept cells keep row-major order."""
        b = np.ascontiguousarray(bc, dtype=np.int32)
        h = ctypes.c_void_p()
        i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
        i, j = i.ravel(), j.ravel()
        if keep is None:
            _check(_L.lxw_mesh_create_cart(nx, ny, x0, x1, y0, y1, _ip(b), ctypes.byref(h)))
        else:
            k = np.ascontiguousarray(np.asarray(keep).reshape(-1) != 0, dtype=np.uint8)
            if k.size != nx * ny:
                raise ValueError("keep needs nx * ny flags")
            _check(_L.lxw_mesh_create_cart_masked(nx, ny, x0, x1, y0, y1, _ip(b),
                                                  k.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), int(wall_bc),
                                                  ctypes.byref(h)))
            i, j = i[k != 0], j[k != 0]
        xs = np.linspace(x0, x1, nx + 1)
        ys = np.linspace(y0, y1, ny + 1)
        v = np.stack([np.stack([xs[i], ys[j]], 1), np.stack([xs[i + 1], ys[j]], 1),
                      np.stack([xs[i + 1], ys[j + 1]], 1), np.stack([xs[i], ys[j + 1]], 1)], 1)
        return Mesh(h, QUAD, v)

    @staticmethod
    def tri(xy, tri, bnd=None, period=None):
        xy = np.ascontiguousarray(xy, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        b = np.ascontiguousarray(bnd, dtype=np.int32) if bnd is not None else None
        p = np.ascontiguousarray(period, dtype=np.float64) if period is not None else None
        h = ctypes.c_void_p()
        _check(_L.lxw_mesh_create_tri(len(xy), _dp(xy), len(tri), _ip(tri), _ip(b) if b is not None else None,
                                      _dp(p) if p is not None else None, ctypes.byref(h)))
        return Mesh(h, TRI, xy[tri])

    @staticmethod
    def tet(xyz, tet, bnd=None, period=None):
        """Tetrahedral P2 mesh: nodes xyz (n x 3), positively oriented tetrahedra (n_tet x 4),
        boundary codes per (tetrahedron, face k opposite vertex k), period (3 lengths)."""
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tet = np.ascontiguousarray(tet, dtype=np.int32)
        b = np.ascontiguousarray(bnd, dtype=np.int32) if bnd is not None else None
        p = np.ascontiguousarray(period, dtype=np.float64) if period is not None else None
        h = ctypes.c_void_p()
        _check(_L.lxw_mesh_create_tet(len(xyz), _dp(xyz), len(tet), _ip(tet), _ip(b) if b is not None else None,
                                      _dp(p) if p is not None else None, ctypes.byref(h)))
        return Mesh(h, TET, xyz[tet])

    def quad_points(self, degree=2):
        """Physical coordinates of the interior quadrature points of every element (N x n x dim)."""
        xi, w, phi = refelem_info(self.kind, degree)
        v = self.verts
        if self.kind == LINE:
            return v[:, 0, None, :] + 0.5 * (xi[None, :, :] + 1.0) * (v[:, 1, None, :] - v[:, 0, None, :])
        if self.kind == TET:
            return v[:, 0, None, :] + sum(xi[None, :, a, None] * (v[:, a + 1, None, :] - v[:, 0, None, :]) for a in range(3))
        if self.kind == TRI:
            return v[:, 0, None, :] + xi[None, :, 0, None] * (v[:, 1, None, :] - v[:, 0, None, :]) \
                + xi[None, :, 1, None] * (v[:, 2, None, :] - v[:, 0, None, :])
        return v[:, 0, None, :] + 0.5 * (xi[None, :, 0, None] + 1) * (v[:, 1, None, :] - v[:, 0, None, :]) \
            + 0.5 * (xi[None, :, 1, None] + 1) * (v[:, 3, None, :] - v[:, 0, None, :])

    def project(self, vals, degree=2):
        """L2 projection of point values at quad_points(degree) (N x n x V) onto the documented basis,
        with the library's quadrature tables: Q_l = sum_m w_m f(x_m) phi_l(x_m)."""
        xi, w, phi = refelem_info(self.kind, degree)
        return np.einsum("m,nmv,ml->nvl", w, np.asarray(vals, dtype=np.float64), phi)


class _Ops:
    """Calls shared by a solver and the solver that runs a batch."""

    def run_steps(self, n):
        _check(_L.lxw_run_steps(self._sh(), n))

    def sync(self):
        _check(_L.lxw_sync(self._sh()))

    def set_timing(self, on=True):
        _check(_L.lxw_set_timing(self._sh(), int(on)))

    def kernel_times(self):
        ms = np.zeros(K_COUNT)
        n = np.zeros(K_COUNT, dtype=np.int64)
        _check(_L.lxw_kernel_times(self._sh(), _dp(ms), n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return {KERNEL_NAMES[k]: (float(ms[k]), int(n[k])) for k in range(K_COUNT)}

    def set_graph(self, on=True):
        _check(_L.lxw_set_graph(self._sh(), int(on)))

    @staticmethod
    def _tune_dict(t):
        d = {KERNEL_NAMES[k]: int(t.block[k]) for k in range(K_COUNT)}
        d["persistent"] = int(t.persistent)
        return d

    def get_tune(self):
        t = Tune()
        _check(_L.lxw_get_tune(self._sh(), ctypes.byref(t)))
        return self._tune_dict(t)

    def set_tune(self, blocks):
        """blocks: {kernel name: workgroup size} for any of the tunable kernels, and "persistent"
        (batches: 0, or the persistent kernel's workgroup size)."""
        t = Tune()
        _check(_L.lxw_get_tune(self._sh(), ctypes.byref(t)))
        for name, b in blocks.items():
            if name == "persistent":
                t.persistent = int(b)
            else:
                t.block[KERNEL_NAMES.index(name)] = int(b)
        _check(_L.lxw_set_tune(self._sh(), ctypes.byref(t)))

    def autotune(self, trial_steps=3):
        t = Tune()
        _check(_L.lxw_autotune(self._sh(), trial_steps, ctypes.byref(t)))
        return self._tune_dict(t)

    def set_indicator(self, ind, tau_lo=0.0, tau_hi=1.0):
        """Learned detection for the shock-capturing limiter (None: plain everywhere)."""
        self._ind = ind  # the indicator must outlive its use
        _check(_L.lxw_solver_set_indicator(self._sh(), ind.h if ind is not None else None, tau_lo, tau_hi))

    def indicator_decisions(self, flags=True):
        """(counts of skipped / plain / flagged decisions since set_indicator, last decision per
        element in the caller's order; for a batch, the meshes' caller orders one after another)."""
        c = np.zeros(3, dtype=np.int64)
        f = np.zeros(self.n_elem, dtype=np.uint8) if flags else None
        _check(_L.lxw_indicator_decisions(self._sh(), c.ctypes.data_as(ctypes.c_void_p),
                                          f.ctypes.data_as(ctypes.c_void_p) if flags else None))
        return c, f


class Solver(_Ops):
    def __init__(self, mesh, stream=None, **params):
        self.mesh = mesh
        self.params = default_params(**params)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        _check(_L.lxw_solver_create(mesh.h, ctypes.byref(self.params), ctypes.c_void_p(stream.cuda_stream),
                                    ctypes.byref(h)))
        self.h = h

    def __del__(self, _destroy=_L.lxw_solver_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def _sh(self):
        return self.h

    @property
    def n_elem(self):
        return self.mesh.N

    @property
    def ML(self):
        return n_modes(self.mesh.kind, self.params.degree)

    @property
    def shape(self):
        return (self.mesh.N, self.mesh.V, self.ML)

    def set_state(self, Q, t0=0.0, checked=True):
        extra = 0 if checked else STATE_UNCHECKED
        if isinstance(Q, torch.Tensor) and Q.is_cuda:
            assert Q.dtype == torch.float64 and Q.is_contiguous() and tuple(Q.shape) == self.shape
            _check(_L.lxw_set_state(self.h, ctypes.c_void_p(Q.data_ptr()), t0, DEVICE_PTR | extra))
        else:
            Q = np.ascontiguousarray(Q, dtype=np.float64)
            assert Q.shape == self.shape, (Q.shape, self.shape)
            _check(_L.lxw_set_state(self.h, Q.ctypes.data_as(ctypes.c_void_p), t0, HOST_PTR | extra))

    def get_state(self, out=None):
        t = ctypes.c_double(0.0)
        if isinstance(out, torch.Tensor) and out.is_cuda:
            _check(_L.lxw_get_state(self.h, ctypes.c_void_p(out.data_ptr()), ctypes.byref(t), DEVICE_PTR))
            return out, t.value
        Q = np.zeros(self.shape)
        _check(_L.lxw_get_state(self.h, Q.ctypes.data_as(ctypes.c_void_p), ctypes.byref(t), HOST_PTR))
        return Q, t.value

    def step(self, T=float("inf")):
        dt = ctypes.c_double(0.0)
        _check(_L.lxw_step(self.h, T, ctypes.byref(dt)))
        return dt.value

    def advance(self, T, max_steps=2**62):
        st = Stats()
        _check(_L.lxw_advance(self.h, T, max_steps, ctypes.byref(st)))
        return st

    def set_debug(self, on=True):
        _check(_L.lxw_set_debug(self.h, int(on)))

    def collect(self):
        """Features [N][48] (float32) and the pending shock-capturing limiter's factor [N]."""
        X = np.zeros((self.mesh.N, NFEAT), dtype=np.float32)
        th = np.zeros(self.mesh.N)
        _check(_L.lxw_indicator_collect(self.h, X.ctypes.data_as(ctypes.c_void_p), th.ctypes.data_as(ctypes.c_void_p),
                                        HOST_PTR))
        return X, th

    def stage(self, stage):
        m = self.mesh
        shapes = {STAGE_QLIM: self.shape, STAGE_QUPD: self.shape, STAGE_VOL: self.shape, STAGE_THETA: (m.N,),
                  STAGE_THETA_SC: (m.N,), STAGE_FLXW: (m.N, m.K, m.V), STAGE_FLXF: (m.N, m.K, m.V),
                  STAGE_C: (m.N, m.K), STAGE_LAME: (m.N, m.K), STAGE_SDT: (2,)}
        out = np.zeros(shapes[stage])
        _check(_L.lxw_debug_stage(self.h, stage, _dp(out)))
        return out


NFEAT, NPARAM = 48, 7361
IND_NOALLOC_MAX = 8192  # LXW_IND_NOALLOC_MAX


def _dev(a, dtype):
    """A contiguous device tensor of dtype holding a (numpy array or tensor)."""
    if isinstance(a, torch.Tensor):
        return a.to(device="cuda", dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype).contiguous()


class Indicator:
    """Learned troubled-cell indicator (lxw_indicator_*): inference, gradients and training run in
    the library's kernels on this object's stream; arrays are passed as device tensors."""

    def __init__(self, params, stream=None):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.shape == (NPARAM,)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        _check(_L.lxw_indicator_create(p.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(stream.cuda_stream),
                                       ctypes.byref(h)))
        self.h = h

    def __del__(self, _destroy=_L.lxw_indicator_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def params(self):
        p = np.zeros(NPARAM, dtype=np.float32)
        _check(_L.lxw_indicator_get_params(self.h, p.ctypes.data_as(ctypes.c_void_p)))
        return p

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        _check(_L.lxw_indicator_set_params(self.h, p.ctypes.data_as(ctypes.c_void_p)))

    def save(self, path):
        _check(_L.lxw_indicator_save(self.h, str(path).encode()))

    def load(self, path):
        _check(_L.lxw_indicator_load(self.h, str(path).encode()))

    def predict(self, X):
        Xd = _dev(X, torch.float32)
        n = Xd.shape[0]
        p = torch.zeros(n, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        _check(_L.lxw_indicator_predict(self.h, ctypes.c_void_p(Xd.data_ptr()), n, ctypes.c_void_p(p.data_ptr())))
        return p.cpu().numpy()

    def grad(self, X, y, w_pos=1.0, w_neg=1.0):
        Xd, yd = _dev(X, torch.float32), _dev(y, torch.float32)
        g = np.zeros(NPARAM, dtype=np.float32)
        loss = ctypes.c_double(0.0)
        torch.cuda.synchronize()
        _check(_L.lxw_indicator_grad(self.h, ctypes.c_void_p(Xd.data_ptr()), ctypes.c_void_p(yd.data_ptr()),
                                     Xd.shape[0], w_pos, w_neg, g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(loss)))
        return g, loss.value

    def grad_noalloc(self, X, y, grad, loss=None, w_pos=1.0, w_neg=1.0):
        """lxw_indicator_grad_noalloc: X (n x 48), y (n), grad (NPARAM) and loss (1, or None) are
        contiguous float32 CUDA tensors of the caller; enqueued on the indicator's stream without
        waiting."""
        for t in (X, y, grad) + ((loss,) if loss is not None else ()):
            assert isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
        n = X.shape[0]
        assert X.shape == (n, NFEAT) and y.shape == (n,) and grad.shape == (NPARAM,)
        _check(_L.lxw_indicator_grad_noalloc(self.h, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(y.data_ptr()), n,
                                             w_pos, w_neg, ctypes.c_void_p(grad.data_ptr()),
                                             ctypes.c_void_p(loss.data_ptr()) if loss is not None else None))

    def train(self, X, y, order, batch, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, w_pos=1.0, w_neg=1.0):
        Xd, yd = _dev(X, torch.float32), _dev(y, torch.float32)
        od = _dev(order, torch.int32)
        n_updates = od.shape[0] // batch
        hp = Adam(lr, beta1, beta2, eps, w_pos, w_neg)
        loss = ctypes.c_double(0.0)
        torch.cuda.synchronize()
        _check(_L.lxw_indicator_train(self.h, ctypes.c_void_p(Xd.data_ptr()), ctypes.c_void_p(yd.data_ptr()),
                                      Xd.shape[0], ctypes.c_void_p(od.data_ptr()), n_updates, batch, ctypes.byref(hp),
                                      ctypes.byref(loss)))
        return loss.value


class Batch(_Ops):
    """Independent meshes of one kind advanced together (lxw_batch_*): per-mesh s, dt and t."""

    def __init__(self, meshes, stream=None, **params):
        self.meshes = list(meshes)
        self.params = default_params(**params)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        arr = (ctypes.c_void_p * len(self.meshes))(*[m.h.value if isinstance(m.h, ctypes.c_void_p) else m.h
                                                      for m in self.meshes])
        h = ctypes.c_void_p()
        _check(_L.lxw_batch_create(len(self.meshes), arr, ctypes.byref(self.params),
                                   ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self.h = h

    def __del__(self, _destroy=_L.lxw_batch_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def _sh(self):
        return _L.lxw_batch_solver(self.h)

    @property
    def n_elem(self):
        return sum(m.N for m in self.meshes)

    def shape(self, i):
        m = self.meshes[i]
        return (m.N, m.V, m.ML)

    def set_state(self, i, Q, t0=0.0, checked=True):
        Q = np.ascontiguousarray(Q, dtype=np.float64)
        assert Q.shape == self.shape(i), (Q.shape, self.shape(i))
        _check(_L.lxw_batch_set_state(self.h, i, Q.ctypes.data_as(ctypes.c_void_p), t0,
                                      HOST_PTR | (0 if checked else STATE_UNCHECKED)))

    def get_state(self, i):
        t = ctypes.c_double(0.0)
        Q = np.zeros(self.shape(i))
        _check(_L.lxw_batch_get_state(self.h, i, Q.ctypes.data_as(ctypes.c_void_p), ctypes.byref(t), HOST_PTR))
        return Q, t.value

    def advance_steps(self, n):
        _check(_L.lxw_batch_advance_steps(self.h, n))

    def stats(self, i):
        st = Stats()
        _check(_L.lxw_batch_stats(self.h, i, ctypes.byref(st)))
        return st
