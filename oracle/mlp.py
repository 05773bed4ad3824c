"""TEST INFRASTRUCTURE ONLY -- FP64 CPU reference of the learned troubled-cell indicator.

The paper detects troubled cells with the shock-capturing limiter it cites (Sec. 1.5 Step 5,
Sec. 4.1).  The learned form replaces only that detection: a small multilayer perceptron maps
normalised modal coefficients of a triangle and its three edge neighbours to the probability that
the limiter acts on the triangle; the positivity limiters of Secs. 3.1-3.3 are untouched.  This
module is the plain float64 statement of that network and of its training loss, written out
layer by layer, for the GPU kernels to be checked against.  Only the tests use it.

Features (48 per triangle): cells c = (i, n_0, n_1, n_2), n_k the neighbour across local edge k
(i itself where edge k is on the boundary); variables rho and E; for each variable the 24 values
Q[c][var][l] (l = 0..5, cell-major), with the centre cell's average subtracted from the four
mode-1 entries, divided by (max |value| + delta_i + 1e-6 |centre average| + 1e-30), where
delta_i = alpha0 h_i^1.5 is the shock-capturing limiter's own relaxation of its bounds (h_i =
sqrt(2 |T_i|)).  The floor carries the magnitude the limiter's decision depends on: variations far
below delta_i (which the limiter never acts on) give features near zero, variations far above it
give their normalised shape; and a uniform region's round-off is never normalised to unit size.
Feature index = var * 24 + c * 6 + l.

Network: 48 -> 64 (ReLU) -> 64 (ReLU) -> 1 (sigmoid).  Parameters in one flat vector:
W1[48][64], b1[64], W2[64][64], b2[64], w3[64], b3 (7,361 values).
Loss over a batch: class-weighted binary cross-entropy
    L = -(1/n) sum_i [ w_pos y_i log p_i + w_neg (1 - y_i) log(1 - p_i) ].
"""
import numpy as np

N_IN, N_H = 48, 64
SIZES = [("W1", (N_IN, N_H)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)), ("w3", (N_H,)), ("b3", ())]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    """Flat parameter vector -> dict of arrays (views)."""
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def tri_neighbours(tri):
    """Neighbour of every triangle across local edge k (vertices k, k+1), -1 on the boundary,
    found by matching vertex pairs."""
    tri = np.asarray(tri)
    nb = -np.ones(tri.shape, dtype=np.int64)
    seen = {}
    for t in range(len(tri)):
        for k in range(3):
            a, b = int(tri[t, k]), int(tri[t, (k + 1) % 3])
            key = (min(a, b), max(a, b))
            if key in seen:
                t2, k2 = seen.pop(key)
                nb[t, k], nb[t2, k2] = t2, t
            else:
                seen[key] = (t, k)
    return nb


def tri_delta(xy, tri, alpha0=500.0):
    """delta_i = alpha0 h_i^1.5 with h_i = sqrt(2 |T_i|)."""
    a = np.asarray(xy, dtype=np.float64)[np.asarray(tri)]
    area = 0.5 * np.abs((a[:, 1, 0] - a[:, 0, 0]) * (a[:, 2, 1] - a[:, 0, 1])
                        - (a[:, 1, 1] - a[:, 0, 1]) * (a[:, 2, 0] - a[:, 0, 0]))
    return alpha0 * np.sqrt(2.0 * area) ** 1.5


def features(Q, nb, delta):
    """48 features per triangle from modal coefficients Q[N][4][6], neighbours nb[N][3] and the
    limiter relaxation delta[N]."""
    N = Q.shape[0]
    cells = np.concatenate([np.arange(N)[:, None], np.where(nb >= 0, nb, np.arange(N)[:, None])], axis=1)
    F = np.zeros((N, N_IN))
    for vi, var in enumerate((0, 3)):
        vals = Q[cells, var, :].copy()            # N x 4 x 6
        vals[:, :, 0] -= Q[:, var, 0][:, None]    # averages relative to the centre cell
        vals = vals.reshape(N, 24)
        scale = np.abs(vals).max(axis=1) + delta + 1e-6 * np.abs(Q[:, var, 0]) + 1e-30
        F[:, vi * 24:(vi + 1) * 24] = vals / scale[:, None]
    return F


def bf16_round(x):
    """Round float64 values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(theta, X, bf16=False):
    """Probabilities p[n].  With bf16=True the inputs, weights and hidden activations are rounded
    to bfloat16 before each product (the inference kernel's number format); sums stay exact-ish
    (float64 here)."""
    P = unpack(np.asarray(theta, dtype=np.float64))
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    a1 = r(X) @ r(P["W1"]) + P["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = r(h1) @ r(P["W2"]) + P["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ P["w3"] + P["b3"]
    return 1.0 / (1.0 + np.exp(-z))


def loss(theta, X, y, w_pos, w_neg):
    p = forward(theta, X)
    y = np.asarray(y, dtype=np.float64)
    return float(-np.mean(w_pos * y * np.log(p) + w_neg * (1.0 - y) * np.log(1.0 - p)))


def grad(theta, X, y, w_pos, w_neg):
    """Gradient of loss() with respect to the flat parameter vector, by the chain rule written
    out layer by layer (reverse order)."""
    P = unpack(np.asarray(theta, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = len(X)
    a1 = X @ P["W1"] + P["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ P["W2"] + P["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ P["w3"] + P["b3"]
    p = 1.0 / (1.0 + np.exp(-z))
    # dL/dz for L_i = -(w_pos y log p + w_neg (1-y) log(1-p)), p = sigmoid(z)
    dz = (w_pos * y * (p - 1.0) + w_neg * (1.0 - y) * p) / n
    g = {}
    g["w3"] = h2.T @ dz
    g["b3"] = np.array(dz.sum())
    dh2 = np.outer(dz, P["w3"])
    da2 = dh2 * (a2 > 0)
    g["W2"] = h1.T @ da2
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ P["W2"].T
    da1 = dh1 * (a1 > 0)
    g["W1"] = X.T @ da1
    g["b1"] = da1.sum(axis=0)
    return np.concatenate([np.ravel(g[name]) for name, _ in SIZES])


def adam(theta, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) of the flat parameters; t counts updates from 1."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
