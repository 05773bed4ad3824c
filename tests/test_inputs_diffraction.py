"""The shock-diffraction domains of Sec. 4 (block step, 120-degree wedge) as the input generator
builds them: the domain filled exactly, boundary tags of the right lengths, triangle counts near
the paper's (126,018 and 122,046), counter-clockwise triangles, and the shock where the paper
places it."""
import numpy as np
import pytest

from paper_1601_08145_amd import inputs as I


@pytest.mark.parametrize("kind,n_paper,wall", [("step", 126018, 1.0 + 6.0),
                                              ("wedge", 122046, 3.4 + float(np.hypot(3.4, 6.0)))])
def test_diffraction_domain(kind, n_paper, wall):
    xy, tri, tags = I.diffraction_domain(kind, n_paper, 0)
    assert abs(len(tri) - n_paper) < 0.01 * n_paper
    a = xy[tri]
    cross = (a[:, 1, 0] - a[:, 0, 0]) * (a[:, 2, 1] - a[:, 0, 1]) - (a[:, 1, 1] - a[:, 0, 1]) * (a[:, 2, 0] - a[:, 0, 0])
    assert np.all(cross > 0)
    solid = I.DIFFRACTION[kind]["solid"]
    sx, sy = np.array(solid).T
    solid_area = 0.5 * abs(np.dot(sx, np.roll(sy, -1)) - np.dot(sy, np.roll(sx, -1)))
    assert 0.5 * cross.sum() == pytest.approx(13.0 * 11.0 - solid_area, rel=1e-12)
    length = {}
    for k in range(3):
        seg = np.linalg.norm(xy[tri[:, (k + 1) % 3]] - xy[tri[:, k]], axis=1)
        for t in (0, 1, 2):
            length[t] = length.get(t, 0.0) + seg[tags[:, k] == t].sum()
    # inflow: x = 0 above the solid (5 long); wall: the solid's surface; the rest transparent
    assert length[0] == pytest.approx(5.0, rel=1e-12)
    assert length[2] == pytest.approx(wall, rel=1e-12)
    assert length[1] == pytest.approx(2 * 13.0 + 11.0 - (1.0 if kind == "step" else 0.0), rel=1e-12)
    # every boundary edge carries a tag, every interior edge -1
    e = np.concatenate([np.sort(np.stack([tri[:, k], tri[:, (k + 1) % 3]], 1), 1) for k in range(3)], 0)
    _, inv, cnt = np.unique(e[:, 0].astype(np.int64) * len(xy) + e[:, 1], return_inverse=True, return_counts=True)
    assert np.array_equal(cnt[inv] == 1, tags.T.ravel() >= 0)


@pytest.mark.parametrize("kind", ["step", "wedge"])
def test_diffraction_state(kind):
    xy, tri, tags = I.diffraction_domain(kind, 20000, 1)
    Q, inflow = I.diffraction_state(xy, tri, kind)
    spec = I.DIFFRACTION[kind]
    pre, post = I.mach_shock_states(spec["mach"])
    c = xy[tri].mean(axis=1)
    h = np.sqrt(2.0 * 137.0 / len(tri))
    ahead = c[:, 0] > spec["x_shock"] + h
    behind = c[:, 0] < spec["x_shock"] - h
    assert behind.any() and ahead.any()
    assert np.allclose(Q[ahead, 0, 0], pre[0]) and np.allclose(Q[behind, 0, 0], post[0])
    assert np.allclose(Q[:, :, 1:], 0.0)
    assert inflow[0] == pytest.approx(post[0])


def test_diffraction_cartesian_step():
    """The block step on the paper's 390 x 330 Cartesian mesh (h = 1/30): the 30 x 180 cells of the
    solid removed, the domain's area filled exactly, the shock on the cell face x = 1 with the
    post-shock state behind it, and the same counts in the oracle's mesh."""
    import oracle as O
    nx, ny, box, bc, keep, Q0, inflow = I.diffraction_cart()
    assert (nx, ny) == (390, 330) and nx * ny - keep.sum() == 30 * 180
    M = O.Mesh.cart(nx, ny, *box, bc, keep=keep, wall_bc=O.BC_REFLECTIVE)
    assert M.N == len(Q0) == 123300 and M.area.sum() == pytest.approx(13.0 * 11.0 - 6.0, rel=1e-12)
    # edges: 4 per cell, the boundary ones counted once (walls 180 + 30, inflow 150, x-high 330,
    # y-low 360, y-high 390)
    assert M.E == (4 * M.N + 210 + 150 + 330 + 360 + 390) // 2
    assert (M.nbr < 0).sum() == 210 + 150 + 330 + 360 + 390
    pre, post = I.mach_shock_states(5.09)
    cons = I.prim_to_cons(np.stack([pre, post]), 1.4)
    jj, ii = np.nonzero(keep.reshape(ny, nx))
    behind = ii < 30
    assert np.allclose(Q0[behind, :, 0], cons[1]) and np.allclose(Q0[~behind, :, 0], cons[0])
    assert np.all(jj[behind] >= 180) and np.allclose(inflow, cons[1]) and np.all(Q0[:, :, 1:] == 0)
