"""GPU tests of the batched form, graph replay and launch-shape tuning (through the C interface).

A batch concatenates independent meshes; each mesh keeps its own wave speed, time step and time,
and must evolve exactly as a single-mesh solver of that mesh does (same kernels, same arithmetic,
so bit for bit).  Graph replays are checked against eager launches with the program's own eager
work and synchronisations between replays; tuning must leave the state untouched and change no
result bit.  One step of batched meshes is also compared with the FP64 oracle."""
import os

import numpy as np
import pytest

import oracle as O
from paper_1601_08145_amd import inputs as I
from tests.helpers import rel_l1

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_1601_08145_amd import lxw
    return lxw


def per_var_rel_l1(a, b):
    return max(rel_l1(a[:, v], b[:, v]) for v in range(a.shape[1]))


def small_batch(L, sizes=(9, 14, 6, 21, 11), seed=3):
    """Uneven vortex + shock meshes (lattice sides `sizes`), shared kernel launches."""
    cases = [I.batch_case(n, seed * 1000 + b) for b, n in enumerate(sizes)]
    meshes = [L.Mesh.tri(xy, tri) for xy, tri, _ in cases]
    return cases, meshes


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_matches_single_solvers_bitwise(L, prec):
    print(f"[gpu] batch vs single solvers, precision {prec}", flush=True)
    cases, meshes = small_batch(L)
    B = L.Batch(meshes, precision=prec)
    for b, (_, _, Q) in enumerate(cases):
        B.set_state(b, Q)
    singles = []
    for b, (_, _, Q) in enumerate(cases):
        S = L.Solver(meshes[b], precision=prec)
        S.set_state(Q)
        singles.append(S)
    # three chunks of graph replays with eager read-outs and synchronisations in between
    for chunk in range(3):
        B.advance_steps(4)
        for S in singles:
            for _ in range(4):
                S.step()
        for b, S in enumerate(singles):
            Qb, tb = B.get_state(b)
            Qs, ts = S.get_state()
            st = B.stats(b)
            assert st.steps == 4 * (chunk + 1)
            assert tb == ts, (chunk, b)
            assert np.array_equal(Qb, Qs), (chunk, b, np.abs(Qb - Qs).max())
    # meshes with different wave speeds took different time steps
    ts = [B.stats(b).t for b in range(len(meshes))]
    assert len(set(ts)) > 1


def test_batch_one_step_vs_oracle(L):
    print("[gpu] batch one step vs oracle", flush=True)
    cases, meshes = small_batch(L, sizes=(12, 7, 17), seed=5)
    B = L.Batch(meshes)
    for b, (_, _, Q) in enumerate(cases):
        B.set_state(b, Q)
    B.advance_steps(1)
    for b, (xy, tri, Q) in enumerate(cases):
        Ob = O.Solver(O.Mesh.tri(xy, tri))
        Ob.set_state(Q)
        Ob.step()
        Qo, to = Ob.get_state()
        Qg, tg = B.get_state(b)
        assert tg == pytest.approx(to, rel=1e-11)
        assert per_var_rel_l1(Qg, Qo) <= 1e-12


def test_batch_state_is_per_mesh(L):
    """Setting one mesh's state restarts only that mesh's time and step count."""
    cases, meshes = small_batch(L, sizes=(8, 10))
    B = L.Batch(meshes)
    for b, (_, _, Q) in enumerate(cases):
        B.set_state(b, Q)
    B.advance_steps(3)
    B.set_state(1, cases[1][2], t0=0.5)
    s0, s1 = B.stats(0), B.stats(1)
    assert s0.steps == 3 and s0.t > 0
    assert s1.steps == 0 and s1.t == 0.5
    Q1, t1 = B.get_state(1)
    assert t1 == 0.5 and np.array_equal(Q1, cases[1][2])


def test_batch_errors(L):
    cases, meshes = small_batch(L, sizes=(8, 10))
    with pytest.raises(L.LxwError) as e:
        L.Batch([meshes[0], L.Mesh.line(20, 0, 1, 1, 1)])
    assert e.value.name == "LXW_ERR_ARG"
    with pytest.raises(L.LxwError):
        L.Batch([])
    B = L.Batch(meshes)
    import ctypes
    Q0 = np.ascontiguousarray(cases[0][2])
    assert L.lib().lxw_batch_set_state(B.h, 2, Q0.ctypes.data_as(ctypes.c_void_p), 0.0, 0) == -1
    assert L.lib().lxw_batch_set_state(B.h, -1, Q0.ctypes.data_as(ctypes.c_void_p), 0.0, 0) == -1
    bad = cases[1][2].copy()
    bad[3, 0, 0] = -1.0
    with pytest.raises(L.LxwError) as e:
        B.set_state(1, bad)
    assert e.value.name == "LXW_ERR_STATE" and "element 3" in e.value.msg
    # single-mesh calls refuse the batch's solver
    lib = L.lib()
    assert lib.lxw_set_debug(B._sh(), 1) == -2
    assert lib.lxw_step(B._sh(), 1.0, None) == -2


@pytest.mark.parametrize("prec", [0, 1])
def test_graph_replay_matches_eager(L, prec):
    xy, tri, Q = I.batch_case(25, 77)
    m = L.Mesh.tri(xy, tri)
    res = []
    for graph in (True, False):
        S = L.Solver(m, precision=prec)
        S.set_graph(graph)
        S.set_state(Q)
        for _ in range(3):
            S.run_steps(5)
            S.sync()
            res.append(S.get_state())
    for k in range(3):
        assert np.array_equal(res[k][0], res[3 + k][0]) and res[k][1] == res[3 + k][1]


def test_launch_shapes_change_no_bit(L):
    xy, tri, Q = I.batch_case(30, 78)
    m = L.Mesh.tri(xy, tri)
    out = []
    for shape in (64, 128, 256):
        S = L.Solver(m, precision=1)
        S.set_tune({k: shape for k in ("k_pre", "k_elem", "k_edge", "k_flim", "k_update")})
        S.set_state(Q)
        S.run_steps(6)
        out.append(S.get_state())
    for k in (1, 2):
        assert np.array_equal(out[0][0], out[k][0]) and out[0][1] == out[k][1]
    S = L.Solver(m)
    with pytest.raises(L.LxwError) as e:
        S.set_tune({"k_elem": 96})
    assert e.value.name == "LXW_ERR_ARG"


def test_autotune_leaves_state_and_trajectory(L):
    print("[gpu] autotune", flush=True)
    cases, meshes = small_batch(L, sizes=(30, 12, 45), seed=9)
    ref = L.Batch(meshes, precision=1)
    B = L.Batch(meshes, precision=1)
    for b, (_, _, Q) in enumerate(cases):
        ref.set_state(b, Q)
        B.set_state(b, Q)
    ref.advance_steps(2)
    B.advance_steps(2)
    before = [B.get_state(b) for b in range(3)]
    tune = B.autotune(2)
    assert all(tune[k] in (64, 128, 256) for k in ("k_pre", "k_elem", "k_edge", "k_flim", "k_update"))
    assert tune["persistent"] in (0, 128, 256)
    assert B.get_tune() == tune
    for b in range(3):
        Qb, tb = B.get_state(b)
        assert np.array_equal(Qb, before[b][0]) and tb == before[b][1]
        assert B.stats(b).steps == 2
    ref.advance_steps(5)
    B.advance_steps(5)
    for b in range(3):
        assert np.array_equal(B.get_state(b)[0], ref.get_state(b)[0])


@pytest.mark.skipif(os.environ.get("LXW_SKIP_FULL") == "1", reason="full-size case skipped on request")
def test_full_size_batch_sampled(L):
    """The batched workload at full size (512 meshes, 2k-60k triangles each, FP32-mixed, graph
    replay, the launch shapes the benchmark tunes): after one step, the smallest, the largest and
    a middle mesh against one FP64 oracle step each."""
    print("[gpu] full-size batch: building 512 meshes", flush=True)
    sizes = I.batch_sizes(512, 0)
    work = I.batch_workload_parallel(512, 0)
    meshes = [L.Mesh.tri(xy, tri) for xy, tri, _ in work]
    B = L.Batch(meshes, precision=1)
    for b in range(len(meshes)):
        B.set_state(b, work[b][2])
    B.autotune(1)
    B.advance_steps(1)
    order = np.argsort(sizes)
    for b in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        xy, tri, Q = work[b]
        Ob = O.Solver(O.Mesh.tri(xy, tri))
        Ob.set_state(Q)
        Ob.step()
        Qo, to = Ob.get_state()
        Qg, tg = B.get_state(b)
        err = per_var_rel_l1(Qg, Qo)
        print(f"[gpu]   mesh {b} ({meshes[b].N} triangles): rel L1 {err:.3e}", flush=True)
        assert tg == pytest.approx(to, rel=2e-6)  # FP32-mixed s is rounded up by a relative 2^-21
        assert err <= 1e-6


def test_batch_of_cartesian_meshes(L):
    """The batched form is not specific to triangles: Cartesian Q2 meshes of different sizes and
    boundary kinds (a near-vacuum blast, periodic; random states with walls and inflow) advance
    together exactly as they do alone."""
    specs = [(24, 24, [0, 0, 0, 0], I.sedov_cart_state(24, 24)),
             (17, 11, [3, 1, 2, 2], I.random_modal_state(17 * 11, 2, 9, seed=3, amp=0.3, rough_frac=0.1,
                                                         rough_amp=2.0, p_range=(1e-3, 1)))]
    meshes = [L.Mesh.cart(nx, ny, -1, 1, -1, 1, bc) for nx, ny, bc, _ in specs]
    B = L.Batch(meshes, precision=1, inflow=[1.2, 0.5, -0.2, 3.0])
    for b, spec in enumerate(specs):
        B.set_state(b, spec[3])
    B.advance_steps(6)
    for b, spec in enumerate(specs):
        S = L.Solver(meshes[b], precision=1, inflow=[1.2, 0.5, -0.2, 3.0])
        S.set_state(spec[3])
        S.run_steps(6)
        Qs, ts = S.get_state()
        Qb, tb = B.get_state(b)
        assert tb == ts and np.array_equal(Qb, Qs)


@pytest.mark.parametrize("prec,speed", [(0, 0), (1, 0), (1, 1)])
def test_batch_masked_meshes_exact_theta(L, prec, speed):
    """Masked Cartesian meshes (the block step's solid, and a box with a removed block and
    periodic sides) with the exact moment-limiter factor, and with either wave speed, advance
    together exactly as they do alone."""
    nx, ny, box, bc, keep, Q0, inflow = I.diffraction_cart(52, 44)
    keep2 = np.ones((20, 26), bool)
    keep2[6:12, 8:14] = False
    Q2 = I.random_modal_state(int(keep2.sum()), 2, 9, seed=9, amp=0.3, rough_frac=0.2, rough_amp=3.0,
                              p_range=(1e-4, 1))
    specs = [(L.Mesh.cart(nx, ny, *box, bc, keep=keep), Q0),
             (L.Mesh.cart(26, 20, 0, 2.6, 0, 2.0, [0, 0, 0, 0], keep=keep2), Q2)]
    kw = dict(precision=prec, theta_exact=1, wave_speed=speed, inflow=list(inflow))
    B = L.Batch([m for m, _ in specs], **kw)
    for b, (_, Q) in enumerate(specs):
        B.set_state(b, Q)
    B.advance_steps(8)
    for b, (m, Q) in enumerate(specs):
        S = L.Solver(m, **kw)
        S.set_state(Q)
        S.run_steps(8)
        Qs, ts = S.get_state()
        Qb, tb = B.get_state(b)
        assert tb == ts and np.array_equal(Qb, Qs), (b, np.abs(Qb - Qs).max())


def test_batch_with_learned_indicator(L):
    """The learned indicator on a batch of triangle meshes: the same decisions and the same states
    as each mesh's own solver with that indicator, bit for bit; the batch's decision flags follow
    the meshes' caller orders one after another."""
    print("[gpu] batch with the learned indicator vs single solvers", flush=True)
    cases, meshes = small_batch(L, sizes=(9, 14, 6, 21), seed=7)
    ind = L.Indicator(I.mlp_init(21))
    # thresholds at the median of this network's outputs on these states, so both decisions occur
    ps = []
    for b, (_, _, Q) in enumerate(cases):
        S = L.Solver(meshes[b], precision=1)
        S.set_state(Q)
        S.step()
        X, _ = S.collect()
        ps.append(ind.predict(X))
    tau = float(np.median(np.concatenate(ps)))
    tau_hi = min(1.0, tau + 0.1)
    B = L.Batch(meshes, precision=1)
    for b, (_, _, Q) in enumerate(cases):
        B.set_state(b, Q)
    B.set_indicator(ind, tau, tau_hi)
    singles = []
    for b, (_, _, Q) in enumerate(cases):
        S = L.Solver(meshes[b], precision=1)
        S.set_state(Q)
        S.set_indicator(ind, tau, tau_hi)
        singles.append(S)
    B.advance_steps(5)
    for S in singles:
        S.run_steps(5)
    cb, fb = B.indicator_decisions()
    dec = [S.indicator_decisions() for S in singles]
    assert np.array_equal(fb, np.concatenate([f for _, f in dec]))
    assert np.array_equal(cb, np.sum([c for c, _ in dec], axis=0))
    assert cb[0] > 0 and cb[1] + cb[2] > 0
    for b, S in enumerate(singles):
        Qb, tb = B.get_state(b)
        Qs, ts = S.get_state()
        assert tb == ts and np.array_equal(Qb, Qs), (b, np.abs(Qb - Qs).max())


def _kind_batch(L, kind, seed):
    """A batch of three uneven meshes of one element kind with rough random states."""
    meshes, states = [], []
    for b, n in enumerate((9, 17, 5)):
        if kind == "tri":
            xy, tri, Q = I.batch_case(n + 4, seed * 100 + b)
            meshes.append(L.Mesh.tri(xy, tri))
            states.append(Q)
        elif kind == "cart":
            meshes.append(L.Mesh.cart(n, n + 2, 0, 1, 0, 1, [0, 0, 1, 1]))
            states.append(I.random_modal_state(n * (n + 2), 2, 9, seed=seed + b, amp=0.3, rough_frac=0.1))
        else:
            meshes.append(L.Mesh.line(4 * n, 0, 1, L.BC_TRANSPARENT, L.BC_REFLECTIVE))
            states.append(I.random_modal_state(4 * n, 1, 3, seed=seed + b, amp=0.3, rough_frac=0.1))
    return meshes, states


PERSISTENT_OFF = ("the persistent kernel is switched off on line and quadrilateral meshes: on a batch of "
                  "quadrilateral meshes its FP32-mixed form reported LXW_ERR_CFL in its first step (FP64 "
                  "equal bit for bit), and on a batch of line meshes one run did not finish; the cause is "
                  "not found")


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind", ["tri", pytest.param("cart", marks=pytest.mark.skip(reason=PERSISTENT_OFF)),
                                  pytest.param("line", marks=pytest.mark.skip(reason=PERSISTENT_OFF))])
def test_persistent_kernel_equals_per_phase_launches(L, kind, prec):
    """The persistent kernel (every phase of every step in one cooperative launch, grid-wide
    barriers between the phases) gives the per-phase launches' results bit for bit, at each of its
    workgroup sizes, over runs longer than one launch's 1024 steps on the smallest batch."""
    print(f"[gpu] persistent kernel, {kind}, precision {prec}", flush=True)
    meshes, states = _kind_batch(L, kind, 5)
    ref = L.Batch(meshes, precision=prec)
    for b, Q in enumerate(states):
        ref.set_state(b, Q)
    ref.advance_steps(7)
    expect = [ref.get_state(b) for b in range(len(meshes))]
    for pw in (128, 256):
        B = L.Batch(meshes, precision=prec)
        B.set_tune({"persistent": pw})
        assert B.get_tune()["persistent"] == pw
        for b, Q in enumerate(states):
            B.set_state(b, Q)
        B.advance_steps(3)
        B.advance_steps(4)
        for b in range(len(meshes)):
            Qb, tb = B.get_state(b)
            assert np.array_equal(Qb, expect[b][0]) and tb == expect[b][1], (pw, b)
            assert B.stats(b).steps == 7
    if prec == 1:
        ref.advance_steps(1100)
        B = L.Batch(meshes, precision=prec)
        B.set_tune({"persistent": 256})
        for b, Q in enumerate(states):
            B.set_state(b, Q)
        B.advance_steps(1107)
        for b in range(len(meshes)):
            assert np.array_equal(B.get_state(b)[0], ref.get_state(b)[0])
    S = L.Solver(meshes[0])
    with pytest.raises(L.LxwError) as e:
        S.set_tune({"persistent": 256})
    assert e.value.name == "LXW_ERR_UNSUPPORTED"


def test_persistent_kernel_refused_off_triangles(L):
    """Batches of line or quadrilateral meshes refuse the persistent kernel (LXW_ERR_UNSUPPORTED)
    and keep the per-phase launches; no kernel runs."""
    for kind in ("cart", "line"):
        meshes, _ = _kind_batch(L, kind, 5)
        B = L.Batch(meshes)
        with pytest.raises(L.LxwError) as e:
            B.set_tune({"persistent": 256})
        assert e.value.name == "LXW_ERR_UNSUPPORTED"
        assert B.get_tune()["persistent"] == 0
