"""GPU: the step's device-side checks (Sec. 3: cell averages stay positive; Sec. 3.2: the
first-order Lax-Friedrichs update is positive) report through the library's error word, name the
offending element in the caller's order (and its mesh in a batch), and leave the solver usable: a
new state steps normally.  Each condition is forced from the host with valid calls:

 * LXW_ERR_CFL: an inflow state (Sec. 2.4) that leaves the domain faster than the global wave speed
   s, which is measured on the elements only, makes Gamma < 0 in the cell next to that side; the
   oracle reports the same code for the same element.
 * LXW_ERR_POSITIVITY / LXW_ERR_NONFINITE: a state set with LXW_STATE_UNCHECKED whose element i has
   a negative density average or a NaN energy average.
"""
import re

import numpy as np
import pytest

import oracle as O
from paper_1601_08145_amd import inputs as I

pytestmark = pytest.mark.gpu

G = 1.4


@pytest.fixture(scope="module")
def L():
    from paper_1601_08145_amd import lxw
    return lxw


def _named(err):
    m = re.search(r"element (-?\d+)", err.msg)
    return int(m.group(1)) if m else None


PRECS = ["FP64", "FP32_MIXED"]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("kind", ["line", "tri"])
def test_cfl_error_from_outgoing_inflow_state(L, kind, prec):
    print(f"[gpu] CFL error, {kind}, {prec}", flush=True)
    rho, u, p = 1.0, -60.0, 1.0
    if kind == "line":
        n = 16
        lm = L.Mesh.line(n, 0, 1, L.BC_INFLOW, L.BC_TRANSPARENT)
        om = O.Mesh.line(n, 0, 1, O.BC_INFLOW, O.BC_TRANSPARENT)
        inflow = [rho, rho * u, 0.0, p / (G - 1) + 0.5 * rho * u * u]
        Q = np.zeros((n, 3, 3))
        Q[:, :, 0] = [1.0, 0.0, 1.0 / (G - 1)]
        bad = 0
    else:
        xy, tri = I.lattice_delaunay(8, 1)
        codes = [L.BC_INFLOW, L.BC_TRANSPARENT, L.BC_TRANSPARENT, L.BC_TRANSPARENT]
        tags = I.boundary_tags(xy, tri, (0, 1, 0, 1), codes)
        lm, om = L.Mesh.tri(xy, tri, tags), O.Mesh.tri(xy, tri, tags)
        inflow = [rho, rho * u, 0.0, p / (G - 1) + 0.5 * rho * u * u]
        Q = np.zeros((len(tri), 4, 6))
        Q[:, :, 0] = [1.0, 0.0, 0.0, 1.0 / (G - 1)]
        bad = np.nonzero((tags == L.BC_INFLOW).any(axis=1))[0]
    S = L.Solver(lm, precision=getattr(L, prec), inflow=inflow)
    S.set_state(Q)
    with pytest.raises(L.LxwError) as ei:
        S.step()
    assert ei.value.code == -7 and ei.value.name == "LXW_ERR_CFL", ei.value
    assert np.isin(_named(ei.value), bad), (ei.value.msg, bad)
    So = O.Solver(om, inflow=inflow)
    So.set_state(Q)
    st, _ = So.step(check=False)
    assert st == -7  # the oracle reports LXW_ERR_CFL too
    if kind == "line":
        assert _named(ei.value) == 0 and O.lib().ora_error_elem(So.h) == 0


def _state(L, kind, seed=3):
    if kind == "line":
        m = L.Mesh.line(40, 0, 1, L.BC_PERIODIC, L.BC_PERIODIC)
        Q = I.random_modal_state(40, 1, 3, seed=seed)
    elif kind == "cart":
        m = L.Mesh.cart(9, 7, 0, 1, 0, 1, [0, 0, 0, 0])
        Q = I.random_modal_state(63, 2, 9, seed=seed)
    else:
        xy, tri = I.lattice_delaunay(10, seed)
        m = L.Mesh.tri(xy, tri)
        Q = I.random_modal_state(len(tri), 2, 6, seed=seed)
    return m, Q


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("kind", ["line", "cart", "tri"])
@pytest.mark.parametrize("what", ["negative_density", "nan_energy"])
def test_state_errors_name_the_element(L, kind, prec, what):
    print(f"[gpu] {what} error, {kind}, {prec}", flush=True)
    m, Q = _state(L, kind)
    i = m.N // 3
    Qb = Q.copy()
    if what == "negative_density":
        Qb[i, 0, 0] = -0.25
        code, name = -5, "LXW_ERR_POSITIVITY"
    else:
        Qb[i, -1, 0] = np.nan
        code, name = -6, "LXW_ERR_NONFINITE"
    S = L.Solver(m, precision=getattr(L, prec))
    with pytest.raises(L.LxwError) as e0:
        S.set_state(Qb)  # the host-side check rejects it
    assert e0.value.code == -4
    S.set_state(Qb, checked=False)
    with pytest.raises(L.LxwError) as ei:
        S.step()
    assert ei.value.code == code and ei.value.name == name, ei.value
    assert _named(ei.value) == i, ei.value.msg
    # usable afterwards: a good state steps normally
    S.set_state(Q)
    S.step()
    Qn, t = S.get_state()
    assert t > 0 and np.all(np.isfinite(Qn))


@pytest.mark.parametrize("prec", PRECS)
def test_batch_error_names_mesh_and_element(L, prec):
    print(f"[gpu] batch error, {prec}", flush=True)
    cases = []
    for seed in (4, 5, 6):
        xy, tri = I.lattice_delaunay(9 + seed, seed)
        cases.append((L.Mesh.tri(xy, tri), I.random_modal_state(len(tri), 2, 6, seed=seed)))
    B = L.Batch([c[0] for c in cases], precision=getattr(L, prec))
    for b, (_, Q) in enumerate(cases):
        B.set_state(b, Q)
    j = 7
    Qb = cases[1][1].copy()
    Qb[j, 0, 0] = -1.0
    B.set_state(1, Qb, checked=False)
    B.advance_steps(1)
    with pytest.raises(L.LxwError) as ei:
        B.sync()
    assert ei.value.code == -5, ei.value
    assert re.search(r"mesh 1, element 7\b", ei.value.msg), ei.value.msg
    B.set_state(1, cases[1][1])
    B.advance_steps(2)
    B.sync()
    assert all(B.stats(b).steps >= 2 for b in range(3))
