"""Benchmark: DG element-updates/s of the LxW-DG step at P2 on 2D triangles (one MI355X).

Workload: 999,698 triangles (Delaunay triangulation of a 708 x 708 jittered point lattice on
[0,1]^2, seed 0, jitter 0.3 h), P2 (6 modes x 4 variables), seeded four-quadrant Riemann data
(rho, p ~ U[0.05, 1], u, v ~ U[-1, 1] per quadrant, cell averages), transparent boundaries, CFL
0.08, plain shock-capturing limiter.  The headline form is FP32-mixed (float32 bulk, float64 cell
averages and flux limiter); the FP64 plain form is timed on the same workload, and the relative L1
difference between the two after the timed steps is reported.

One JSON line on stdout.  Inputs are resident in HBM before the timed region; the timed region is
exactly --steps steps, bracketed by torch.cuda.synchronize().  Per-kernel HIP events recorded
around every launch inside the timed region give the average duration of the dominant kernel
(k_elem) for the roofline entry.  The CPU baseline is the oracle (tests only otherwise) timed on
a bounded sample: one step of the same workload on all host cores.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-fp64]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DG element-updates/s at P2 2D tri; mixed/learned vs FP64 plain at equal L1"

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_FP64_VECTOR_TFLOPS = 78.6

# Algorithmic work of k_elem per triangle (P2), counted from the kernel's arithmetic: Galerkin
# projection of F at 7 points, q / grad q / div F^h / grad div F^h and F_T at 16 points, volume
# term at 7 points, traces at 9 points.  See the design doc (roofline) for the count.
KELEM_FLOPS_PER_ELEM = 15.9e3
# bytes: state in (cell averages f64 4x8 + higher modes 20 x R) + geometry (Jinv 4 R, outward
# normals 6 R, edge slots 3 x 4) + higher modes out (20 x R) + traces out (3 edges x 3 points x
# (q, n.F_T) x 4 variables x R)
def kelem_bytes_per_elem(rsize):
    return 4 * 8 + 20 * rsize + 10 * rsize + 12 + 20 * rsize + 72 * rsize


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def build_workload():
    from paper_1601_08145_amd import inputs as I
    t0 = time.time()
    xy, tri = I.lattice_delaunay(708, 0)
    Q0 = I.averages_to_modal(I.cell_average_state(I.four_quadrant_fn(0), I.tri_sample_points(xy, tri, 2), 1.4), 6)
    log(f"[bench] workload: {len(tri)} triangles, built in {time.time() - t0:.1f} s")
    return xy, tri, Q0


def time_gpu(L, mesh, Q0, precision, steps, warmup, kernel_events=True):
    import torch
    S = L.Solver(mesh, precision=precision)
    S.set_state(Q0)
    S.run_steps(warmup)
    S.sync()
    if kernel_events:
        S.set_timing(True)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t0 = time.perf_counter()
    S.run_steps(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    S.sync()
    ms = e0.elapsed_time(e1)
    kt = S.kernel_times() if kernel_events else {}
    Q, t = S.get_state()
    return {"ms_total": ms, "wall_s": wall, "kernels": kt, "Q": Q, "t": t}


def cpu_baseline(xy, tri, Q0):
    import oracle as O
    m = O.Mesh.tri(xy, tri)
    S = O.Solver(m)
    S.set_state(Q0)
    t0 = time.perf_counter()
    S.step()
    dt = time.perf_counter() - t0
    return {"value": len(tri) / dt, "unit": "element-updates/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"one step of the same {len(tri)}-triangle workload (FP64 oracle, {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-kernel-events", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only copy a float32 buffer of BYTES bytes 3 times (reference for HBM counters)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        n = args.copy_probe // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 4, "copies": 3}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the LxW-DG step here is a "
                          "single-GPU build (multi-GPU sharding is a design note, not implemented)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_1601_08145_amd import lxw as L

    xy, tri, Q0 = build_workload()
    mesh = L.Mesh.tri(xy, tri)
    N = mesh.N

    log(f"[bench] FP32-mixed: {args.warmup} warm-up + {args.steps} timed steps")
    mix = time_gpu(L, mesh, Q0, L.FP32_MIXED, args.steps, args.warmup, not args.no_kernel_events)
    ms_step = mix["ms_total"] / args.steps
    value = N * args.steps / (mix["ms_total"] * 1e-3)
    log(f"[bench]   {ms_step:.3f} ms/step, {value:.4e} element-updates/s")

    out = {"metric": METRIC, "value": value, "unit": "element-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32 (f64 cell averages and flux limiter)", "data": "synthetic",
           "config": {"workload": "2D Euler, P2 triangles, 999,698-triangle Delaunay mesh of a 708^2 lattice "
                                  "jittered 0.3h on [0,1]^2, four-quadrant Riemann data seed 0, transparent "
                                  "boundaries, CFL 0.08, plain shock limiter",
                      "n_elem": N, "n_edge": mesh.E, "precision": "FP32_MIXED"}}

    if mix["kernels"]:
        kt = {k: {"ms_avg": v[0] / max(v[1], 1), "launches": v[1]} for k, v in mix["kernels"].items()}
        out["kernels"] = kt
        kavg = kt["k_elem"]["ms_avg"]
        flops = KELEM_FLOPS_PER_ELEM * N
        achieved = flops / (kavg * 1e-3) / 1e12
        bytes_ = kelem_bytes_per_elem(4) * N
        out["roofline"] = {"kernel": "k_elem", "bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS,
                           "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": None,
                           "kernel_ms": kavg, "flops_per_elem": KELEM_FLOPS_PER_ELEM,
                           "hbm_view": {"achieved_GBs": bytes_ / (kavg * 1e-3) / 1e9, "peak_GBs": PEAK_HBM_GBS,
                                        "frac": bytes_ / (kavg * 1e-3) / 1e9 / PEAK_HBM_GBS,
                                        "bytes_per_elem": kelem_bytes_per_elem(4)}}

    if not args.no_fp64:
        log(f"[bench] FP64 plain: {args.warmup} warm-up + {args.steps} timed steps")
        f64 = time_gpu(L, mesh, Q0, L.FP64, args.steps, args.warmup, False)
        v64 = N * args.steps / (f64["ms_total"] * 1e-3)
        a, b = mix["Q"], f64["Q"]
        rel = max(float(np.abs(a[:, v] - b[:, v]).sum() / np.abs(b[:, v]).sum()) for v in range(4))
        out["fp64_plain"] = {"value": v64, "ms_per_step": f64["ms_total"] / args.steps}
        out["mixed_vs_fp64"] = {"speedup": value / v64, "rel_l1_state_diff": rel,
                                "note": f"states after {args.warmup + args.steps} steps from the same input"}
        log(f"[bench]   FP64 {v64:.4e} element-updates/s; mixed/FP64 {value / v64:.2f}x; rel L1 diff {rel:.2e}")

    if not args.no_cpu_baseline:
        log("[bench] CPU baseline (oracle, one step)")
        out["cpu_baseline"] = cpu_baseline(xy, tri, Q0)
        log(f"[bench]   {out['cpu_baseline']['value']:.4e} element-updates/s on {out['cpu_baseline']['cores']} threads")

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
