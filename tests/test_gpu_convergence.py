"""GPU: accuracy of the library's step on smooth solutions, at mesh sizes past the oracle's
convergence tests (the paper's convergence study, Sec. 4.3.1): Shu's isentropic vortex advected on
periodic Cartesian Q2 and triangle P2 meshes, cell-average density against the exact solution's
cell averages (the oracle's L2 projection of the exact solution, mode 1)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1601_08145_amd import inputs as I
from tests import helpers as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_1601_08145_amd import lxw
    return lxw


def vortex(x, t):
    return H.cons(H.vortex_prim(x[..., 0], x[..., 1], t, period=(10.0, 10.0)))


@pytest.mark.parametrize("kind", ["cart", "tri"])
def test_vortex_convergence(L, kind):
    """FP64: the L1 error of the cell-average density falls at order above 2.5 between the two
    finest meshes (Cartesian 32^2 -> 128^2, triangles on 33^2 -> 129^2 lattices); the FP32-mixed
    form is within 10% of the FP64 error on the coarsest mesh, where the discretisation error is
    far above float32 rounding, and exceeds 1.1 x the FP64 error by at most its rounding floor on
    the others (5e-7; measured 1.5e-7 on Cartesian and 4e-7 on triangle meshes, densities of
    order 1)."""
    T = 0.5
    errs = {L.FP64: [], L.FP32_MIXED: []}
    sizes = [32, 64, 128] if kind == "cart" else [33, 65, 129]
    for n in sizes:
        if kind == "cart":
            lm = L.Mesh.cart(n, n, -5, 5, -5, 5, [0, 0, 0, 0])
            om = O.Mesh.cart(n, n, -5, 5, -5, 5, [O.BC_PERIODIC] * 4)
        else:
            xy, tri = I.lattice_delaunay(n, 3, box=(-5.0, 5.0, -5.0, 5.0), periodic=True)
            tags = I.boundary_tags(xy, tri, (-5, 5, -5, 5), [0, 0, 0, 0])
            lm = L.Mesh.tri(xy, tri, tags, (10.0, 10.0))
            om = O.Mesh.tri(xy, tri, tags, (10.0, 10.0))
        Q0 = om.project(vortex(om.quad_points(), 0.0))
        ref = om.project(vortex(om.quad_points(), T))[:, 0, 0]
        for prec in errs:
            S = L.Solver(lm, precision=prec)
            S.set_state(Q0)
            S.advance(T)
            Q, t = S.get_state()
            assert t == T
            errs[prec].append(float(np.sum(np.abs(Q[:, 0, 0] - ref) * om.area) / om.area.sum()))
    orders = [math.log2(errs[L.FP64][i] / errs[L.FP64][i + 1]) for i in range(len(sizes) - 1)]
    print(f"[gpu] vortex {kind}: L1(rho) FP64 {['%.3e' % e for e in errs[L.FP64]]}, orders "
          f"{['%.2f' % o for o in orders]}; FP32-mixed {['%.3e' % e for e in errs[L.FP32_MIXED]]}", flush=True)
    assert orders[-1] > 2.5
    assert abs(errs[L.FP32_MIXED][0] - errs[L.FP64][0]) <= 0.1 * errs[L.FP64][0]
    for e32, e64 in zip(errs[L.FP32_MIXED], errs[L.FP64]):
        assert e32 <= 1.1 * e64 + 5e-7
