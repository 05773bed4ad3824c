"""Pins of the FP64 CPU reference of the learned indicator (oracle/mlp.py): gradients against
central finite differences, the loss against scikit-learn's log loss, bfloat16 rounding against
torch's conversion, Adam's first step against its closed form, and the features against their
invariances and a hand-computed case."""
import numpy as np
import pytest

from oracle import mlp as M


def he_init(seed):
    g = np.random.default_rng(seed)
    th = np.zeros(M.N_PARAMS)
    P = M.unpack(th)
    P["W1"][:] = g.uniform(-1, 1, P["W1"].shape) * np.sqrt(6.0 / M.N_IN)
    P["W2"][:] = g.uniform(-1, 1, P["W2"].shape) * np.sqrt(6.0 / M.N_H)
    P["w3"][:] = g.uniform(-1, 1, P["w3"].shape) * np.sqrt(6.0 / M.N_H)
    P["b1"][:] = g.uniform(-0.1, 0.1, M.N_H)
    P["b2"][:] = g.uniform(-0.1, 0.1, M.N_H)
    P["b3"][...] = 0.05
    return th


def test_parameter_count():
    assert M.N_PARAMS == 48 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 7361


def test_gradient_matches_central_differences():
    g = np.random.default_rng(1)
    th = he_init(0)
    X = g.uniform(-1, 1, (40, 48))
    y = (g.uniform(0, 1, 40) < 0.3).astype(float)
    wp, wn = 2.5, 0.7
    an = M.grad(th, X, y, wp, wn)
    idx = np.concatenate([g.choice(M.N_PARAMS, 300, replace=False), np.arange(3072, 3136), [M.N_PARAMS - 1]])
    h = 1e-6
    for j in idx:
        e = np.zeros_like(th)
        e[j] = h
        fd = (M.loss(th + e, X, y, wp, wn) - M.loss(th - e, X, y, wp, wn)) / (2 * h)
        assert abs(fd - an[j]) <= 1e-7 + 1e-5 * abs(fd), (j, fd, an[j])


def test_loss_is_log_loss_when_unweighted():
    sk = pytest.importorskip("sklearn.metrics")
    g = np.random.default_rng(2)
    th = he_init(3)
    X = g.uniform(-1, 1, (64, 48))
    y = (g.uniform(0, 1, 64) < 0.5).astype(float)
    p = M.forward(th, X)
    assert M.loss(th, X, y, 1.0, 1.0) == pytest.approx(sk.log_loss(y, p, labels=[0, 1]), rel=1e-12)


def test_forward_special_cases():
    th = np.zeros(M.N_PARAMS)
    M.unpack(th)["b3"][...] = 0.3
    X = np.random.default_rng(4).uniform(-1, 1, (5, 48))
    assert np.allclose(M.forward(th, X), 1 / (1 + np.exp(-0.3)), rtol=0, atol=1e-15)
    # one path: feature 7 -> hidden 2 -> hidden 5 -> output, all weights 1 (ReLU passes positives)
    th = np.zeros(M.N_PARAMS)
    P = M.unpack(th)
    P["W1"][7, 2] = 1.0
    P["W2"][2, 5] = 1.0
    P["w3"][5] = 1.0
    X = np.zeros((3, 48))
    X[:, 7] = [0.5, -0.5, 2.0]
    assert np.allclose(M.forward(th, X), 1 / (1 + np.exp(-np.array([0.5, 0.0, 2.0]))), atol=1e-15)


def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    x = np.random.default_rng(5).standard_normal(10000) * 10.0 ** np.random.default_rng(6).uniform(-5, 5, 10000)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16_round(x), ref)


def test_adam_first_step_closed_form():
    th = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    t1, m, v = M.adam(th, np.zeros(3), np.zeros(3), g, 1, lr=0.01, eps=1e-12)
    # first update: m_hat = g, v_hat = g^2 -> step lr * g / |g|
    assert np.allclose(t1, th - 0.01 * np.sign(g), rtol=0, atol=1e-10)


def test_neighbours_and_hand_computed_features():
    # two triangles sharing the edge (1, 2): local edge 1 of t0 (vertices 1 -> 2) and local edge 1
    # of t1 (vertices 2 -> 1)
    tri = np.array([[0, 1, 2], [3, 2, 1]])
    nb = M.tri_neighbours(tri)
    assert nb.tolist() == [[-1, 1, -1], [-1, 0, -1]]
    Q = np.zeros((2, 4, 6))
    Q[0, 0, :] = [1.0, 0.2, 0.0, 0.0, 0.0, 0.1]
    Q[1, 0, :] = [3.0, 0.0, 0.0, 0.0, 0.0, 0.0]
    Q[0, 3, 0] = 2.0
    Q[1, 3, 0] = 2.0
    F = M.features(Q, nb, np.array([0.25, 0.5]))
    # t0, rho: cells (0, 0, 1, 0): averages 0, 0, 2, 0 relative to 1.0; scale 2 + 0.25 + 1e-6 * 1
    rho = F[0, :24].reshape(4, 6)
    sc = 2.0 + 0.25 + 1e-6
    assert np.allclose(rho[0], np.array([0.0, 0.2, 0, 0, 0, 0.1]) / sc, rtol=1e-14)
    assert np.allclose(rho[2], np.array([2.0, 0, 0, 0, 0, 0]) / sc, rtol=1e-14)
    assert np.allclose(rho[1], rho[0]) and np.allclose(rho[3], rho[0])
    # E is uniform: every feature is 0
    assert np.all(F[:, 24:] == 0.0)


def test_features_bounded_and_magnitude_aware():
    g = np.random.default_rng(7)
    from paper_1601_08145_amd import inputs as I
    xy, tri = I.lattice_delaunay(12, 3)
    nb = M.tri_neighbours(tri)
    delta = M.tri_delta(xy, tri, alpha0=0.5)
    Q = I.random_modal_state(len(tri), 2, 6, seed=4, amp=0.5)
    F = M.features(Q, nb, delta)
    assert np.all(np.abs(F) < 1.0)
    # without a relaxation the normalisation is by the largest value: scale invariant, max 1
    F0 = M.features(Q, nb, 0.0 * delta)
    assert np.allclose(M.features(3.7 * Q, nb, 0.0 * delta), F0, rtol=1e-5, atol=1e-7)
    for vi in range(2):
        assert np.allclose(np.abs(F0[:, vi * 24:(vi + 1) * 24]).max(axis=1), 1.0, rtol=1e-5)
    # variations far below delta give features near zero, far above it their normalised shape
    small = 1e-6 * Q
    small[:, :, 0] += 1.0
    assert np.abs(M.features(small, nb, delta)).max() < 1e-3
    # the tri_delta geometry: h = sqrt(2 |T|) is the lattice spacing of a split unit square
    xs, ts = np.array([[0, 0], [1, 0], [0, 1]], float), np.array([[0, 1, 2]])
    assert M.tri_delta(xs, ts, 500.0)[0] == pytest.approx(500.0)
    # a uniform state plus round-off gives features near zero, not unit-size noise
    U = np.zeros_like(Q)
    U[:, :, 0] = Q[0, :, 0]
    U[:, :, 1:] = 1e-17 * g.standard_normal(U[:, :, 1:].shape)
    assert np.abs(M.features(U, nb, 0.0 * delta)).max() < 1e-9
