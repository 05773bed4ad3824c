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

A second, batched leg advances 512 independent meshes of 2k-60k triangles together (graph replay,
autotuned launch shapes) and is reported under "batched".  A third leg trains the learned
troubled-cell indicator with the library's kernels and compares the learned form with the plain
form ("learned").

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-fp64] [--no-batched]
                 [--no-learned]
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

# MI355X published peaks: HBM3E 8 TB/s; fp32 vector 157.3 TFLOP/s (256 CUs x 2.4 GHz x 128 fp32 FMA
# lanes x 2 flops, counting packed fp32).  This library is built with packed fp32 instructions
# disabled, so the fp32 (and fp64) vector rate its kernels can reach is 64 FMA lanes x 2 flops x 256
# CUs x 2.4 GHz = 78.6 TFLOP/s; roofline fractions are given against the published peak, with the
# non-packed fraction beside it.
PEAK_HBM_GBS = 8000.0
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_VECTOR_NONPACKED_TFLOPS = 78.6
# Algorithmic bytes of one whole step per triangle, FP32 bulk (state of 6 modes x 4 variables read
# and written, 96 B each way, plus the mesh: 3 neighbour ids and orientation 16 B, Jinv and |T|
# 20 B): 96 + 96 + 36 = 228 B.  The minimum a step must move; the kernels' traces, edge records and
# limiter factors are intermediates on top of it.
STEP_BYTES_PER_ELEM = 228

# Arithmetic of k_elem per triangle (P2, FP32-mixed): projection of F at 7 points, q, grad q,
# div F^h, grad div F^h and F_T at 16 points, volume term, traces.  Counted from the kernel's
# executed VALU instructions per wavefront (64 triangles): fp32 FMA x 2 + fp32 add + fp32 mul +
# fp64 FMA x 2 + fp64 add + fp64 mul, divided by 64 (profiles/lxw_kernels_tri_c3_counters.md).
KELEM_FLOPS_PER_ELEM = 9.41e3
# The bound k_elem actually meets: VALU instruction issue.  Executed VALU instructions per wavefront
# of 64 triangles (SQ_INSTS_VALU / SQ_WAVES, same counter file); a wave64 VALU instruction occupies a
# 16-lane SIMD for 4 cycles, and the chip has 256 CUs x 4 SIMDs at 2.4 GHz.
KELEM_VALU_INSTS_PER_WAVE = 5872
VALU_SIMDS, CLOCK_GHZ = 1024, 2.4
# Bytes k_elem must move per triangle (FP32-mixed): cell averages in (4 x f64), higher modes in
# (20 x f32), limiter factor (f64), geometry (Jinv 4 x f32, outward normals 6 x f32, edge slots
# 3 x i32), higher modes out (20 x f32), traces out (3 edges x 3 points x 4 x f32: one record per
# edge side and point, n_out.F_T/2 + (s|n|/2) q).
def kelem_bytes_per_elem(rsize):
    return 4 * 8 + 20 * rsize + 8 + 10 * rsize + 12 + 20 * rsize + 36 * rsize


# HBM traffic of one launch of each step kernel on the 2D triangle workload (FP32-mixed) from
# rocprofv3 counters (FETCH_SIZE x 2 + WRITE_SIZE, scale factors from a copy of known size), valid
# only for the kernel source it was measured on.
TRAFFIC = {"src_sha256": "e2c6f33d22e97d9db911cd1b7a12a36f6a8142f6f385f2e124f4789be58e47d0",
           "bytes_per_launch": {"k_pre": 138976369, "k_elem": 409446605, "k_edge": 381145088,
                                "k_flim": 174059520, "k_update": 399809536}}  # profiles/lxw_kernels_tri_c3_counters.md


def traffic_valid():
    return TRAFFIC["src_sha256"] == kernel_src_hash()


def kernel_src_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("lxw_kernels.hip", "lxw_internal.hpp", "lxw_host.cpp"):  # kernels, layout, element order
        with open(os.path.join(ROOT, "paper_1601_08145_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def build_workload():
    from paper_1601_08145_amd import inputs as I
    t0 = time.time()
    xy, tri = I.lattice_delaunay(708, 0)
    Q0 = I.averages_to_modal(I.cell_average_state(I.four_quadrant_fn(0), I.tri_sample_points(xy, tri, 2), 1.4), 6)
    log(f"[bench] workload: {len(tri)} triangles, built in {time.time() - t0:.1f} s")
    return xy, tri, Q0


def _timed(S, steps):
    import torch
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    S.run_steps(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    S.sync()
    return e0.elapsed_time(e1)


def time_gpu(L, mesh, Q0, precision, steps, warmup, kernel_events=True, kw=None):
    """Two timed regions of `steps` steps each after `warmup` steps: (1) every kernel launched by
    the library with HIP events around each launch (per-kernel durations); (2) the step replayed
    from its HIP graph."""
    S = L.Solver(mesh, precision=precision, **(kw or {}))
    S.set_state(Q0)
    S.run_steps(warmup)
    S.sync()
    S.set_timing(kernel_events)
    if not kernel_events:
        S.set_graph(False)
    ms = _timed(S, steps)
    kt = S.kernel_times() if kernel_events else {}
    S.set_timing(False)
    S.set_graph(True)
    ms_graph = _timed(S, steps)
    Q, t = S.get_state()
    return {"ms_total": ms, "ms_graph": ms_graph, "kernels": kt, "Q": Q, "t": t}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(xy, tri, Q0):
    """The oracle (FP64, OpenMP over elements and edges) on the host cores: steps of the full
    workload on all threads until 10 s have passed (at least two), and one step of a
    200^2-lattice mesh of the same kind on one thread."""
    import oracle as O
    m = O.Mesh.tri(xy, tri)
    S = O.Solver(m)
    S.set_state(Q0)
    t0 = time.perf_counter()
    n_steps = 0
    while n_steps < 2 or time.perf_counter() - t0 < 10.0:
        S.step()
        n_steps += 1
    dt = time.perf_counter() - t0
    cores = O.num_threads()
    from paper_1601_08145_amd import inputs as I
    xs, ts = I.lattice_delaunay(200, 0)
    Qs = I.averages_to_modal(I.cell_average_state(I.four_quadrant_fn(0), I.tri_sample_points(xs, ts, 2), 1.4), 6)
    O.set_num_threads(1)
    S1 = O.Solver(O.Mesh.tri(xs, ts))
    S1.set_state(Qs)
    t1 = time.perf_counter()
    S1.step()
    dt1 = time.perf_counter() - t1
    O.set_num_threads(cores)
    return {"value": len(tri) * n_steps / dt, "unit": "element-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_steps} steps of the same {len(tri)}-triangle workload (FP64 oracle, {dt:.1f} s on "
                      f"{cores} threads)",
            "one_thread": {"value": len(ts) / dt1, "sample": f"one step of a {len(ts)}-triangle mesh of the same "
                                                             f"kind on 1 thread ({dt1:.1f} s)"},
            "cpu_model": cpu_model(), "nproc": os.cpu_count()}


def copy_rate(nbytes=1 << 30, reps=5):
    """Bytes read + written per second of a device-to-device copy of nbytes (fastest of reps): the
    rate a plain streaming kernel reaches, beside which the memory-bound step kernels are read."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1)
        best = t if best is None else min(best, t)
    del a, b
    return 2 * nbytes / (best * 1e-3)


def kelem_roofline(kavg_ms, n_elem, traffic_ok, ms_per_step=None):
    """Roofline of the dominant kernel k_elem (fp32 vector arithmetic) against the published fp32
    peak; with ms_per_step, the whole step's algorithmic bytes against the HBM peak and the counted
    traffic of the step's kernels against those bytes."""
    achieved = KELEM_FLOPS_PER_ELEM * n_elem / (kavg_ms * 1e-3) / 1e12
    issue_ms = KELEM_VALU_INSTS_PER_WAVE * (-(-n_elem // 64)) * 4 / VALU_SIMDS / (CLOCK_GHZ * 1e9) * 1e3
    bytes_ = kelem_bytes_per_elem(4) * n_elem
    traffic = None
    if traffic_ok and traffic_valid():
        traffic = TRAFFIC["bytes_per_launch"]["k_elem"]
    out = {"kernel": "k_elem", "bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS,
           "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": traffic,
           "kernel_ms": kavg_ms, "flops_per_elem": KELEM_FLOPS_PER_ELEM, "units_per_launch": n_elem,
           "frac_of_nonpacked_fp32_peak": achieved / PEAK_VECTOR_NONPACKED_TFLOPS,
           "nonpacked_fp32_peak": PEAK_VECTOR_NONPACKED_TFLOPS,
           "issue_view": {"valu_insts_per_wave": KELEM_VALU_INSTS_PER_WAVE, "waves": -(-n_elem // 64),
                          "issue_ms": issue_ms, "frac": issue_ms / kavg_ms,
                          "note": "VALU issue time of the counted instructions (4 cycles per wave64 "
                                  "instruction, 1024 SIMDs at 2.4 GHz) over the kernel time"},
           "hbm_view": {"achieved_GBs": bytes_ / (kavg_ms * 1e-3) / 1e9, "peak_GBs": PEAK_HBM_GBS,
                        "frac": bytes_ / (kavg_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                        "bytes_per_elem": kelem_bytes_per_elem(4)}}
    if ms_per_step is not None:
        sb = STEP_BYTES_PER_ELEM * n_elem
        step = {"bytes_per_elem": STEP_BYTES_PER_ELEM, "algorithmic_bytes": sb, "ms_per_step": ms_per_step,
                "achieved_GBs": sb / (ms_per_step * 1e-3) / 1e9, "peak_GBs": PEAK_HBM_GBS,
                "frac": sb / (ms_per_step * 1e-3) / 1e9 / PEAK_HBM_GBS}
        if traffic_ok and traffic_valid():
            counted = sum(TRAFFIC["bytes_per_launch"].values())
            step["counted_traffic_bytes"] = counted
            step["counted_over_algorithmic"] = counted / sb
        out["step_hbm"] = step
    return out


def time_batch_graph(B, steps):
    import torch
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    e0.record(stream)
    B.advance_steps(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    B.sync()
    return e0.elapsed_time(e1)


def batched_leg(L, steps, warmup):
    """512 independent triangle meshes (2k-60k triangles, log-uniform), vortex + shock data,
    FP32-mixed, advanced together: graph replay with the default and the autotuned launch shapes,
    eager launches for comparison, and per-kernel times."""
    from paper_1601_08145_amd import inputs as I
    t0 = time.time()
    work = I.batch_workload_parallel(512, 0)
    meshes = [L.Mesh.tri(xy, tri) for xy, tri, _ in work]
    ntot = sum(m.N for m in meshes)
    log(f"[bench] batched: {len(meshes)} meshes, {ntot} triangles, built in {time.time() - t0:.1f} s")
    B = L.Batch(meshes, precision=L.FP32_MIXED)
    for b, (_, _, Q) in enumerate(work):
        B.set_state(b, Q)
    del work
    B.advance_steps(warmup)
    B.sync()
    ms_default = time_batch_graph(B, steps)
    default_tune = B.get_tune()
    tune = B.autotune(3)
    ms_tuned = time_batch_graph(B, steps)
    # A/B of the step's form at the tuned workgroup sizes: one launch per phase replayed from the
    # graph, against the persistent kernel (all phases of all steps in one cooperative launch)
    ab = {}
    for pw in (0, 128, 256):
        B.set_tune(dict(tune, persistent=pw))
        ab["graph" if pw == 0 else f"persistent_{pw}"] = time_batch_graph(B, steps) / steps
    log(f"[bench]   batched form A/B (ms/step): {ab}")
    B.set_tune(dict(tune, persistent=0))
    B.set_graph(False)
    ms_eager = time_batch_graph(B, steps)
    B.set_graph(True)
    B.set_tune(tune)
    B.set_timing(True)
    B.advance_steps(min(steps, 20))
    B.sync()
    kt = {k: {"ms_avg": v[0] / max(v[1], 1), "launches": v[1]} for k, v in B.kernel_times().items()}
    B.set_timing(False)
    value = ntot * steps / (ms_tuned * 1e-3)
    log(f"[bench]   batched {ms_tuned / steps:.3f} ms/step tuned ({tune}), {ms_default / steps:.3f} default, "
        f"{ms_eager / steps:.3f} eager; {value:.4e} element-updates/s")
    return {"workload": "512 independent 2D Euler P2 triangle meshes, 2k-60k triangles each (log-uniform, seed 0), "
                        "jittered-lattice Delaunay on [-5,5]^2, isentropic vortex + random planar shock, "
                        "FP32-mixed, per-mesh dt, the step's form (one launch per phase replayed from a HIP "
                        "graph, or one persistent cooperative kernel) and workgroup sizes autotuned",
            "n_meshes": len(meshes), "n_elem": ntot, "steps": steps, "value": value, "unit": "element-updates/s",
            "ms_per_step": ms_tuned / steps, "tune": tune,
            "persistent_ab_ms_per_step": ab,
            "default_tune": {"tune": default_tune, "ms_per_step": ms_default / steps},
            "eager_launches": {"ms_per_step": ms_eager / steps},
            "kernels": kt, "roofline": kelem_roofline(kt["k_elem"]["ms_avg"], ntot, traffic_ok=False)}


def rel_l1(a, b):
    return max(float(np.abs(a[:, v] - b[:, v]).sum() / np.abs(b[:, v]).sum()) for v in range(a.shape[1]))


def time_steps(L, mesh, Q0, steps, warmup, ind=None, tau=(0.0, 1.0), kw=None):
    """FP32-mixed steps replayed from the graph (timed), then per-kernel events; returns
    (ms per step, kernel averages, final state, decision counts)."""
    S = L.Solver(mesh, precision=L.FP32_MIXED, **(kw or {}))
    S.set_state(Q0)
    if ind is not None:
        S.set_indicator(ind, *tau)
    S.run_steps(warmup)
    S.sync()
    ms = _timed(S, steps)
    S.set_timing(True)
    S.run_steps(steps)  # as many steps again, so that states compare with the other legs' after warmup + 2 steps
    S.sync()
    kt = {k: v[0] / max(v[1], 1) for k, v in S.kernel_times().items()}
    S.set_timing(False)
    Q, _ = S.get_state()
    counts = S.indicator_decisions(False)[0].tolist() if ind is not None else None
    return ms / steps, kt, Q, counts


def learned_leg(L, steps, warmup, c3_mesh, c3_Q0, fp64_Q=None):
    """Train the indicator with the library's kernels on plain runs of the four-quadrant and blast
    families, then run the learned form against the plain form on the 2D triangle workload and on a
    2M-triangle ramp with a Mach 10 shock (outside the training families)."""
    from paper_1601_08145_amd import indicator_train as T, inputs as I
    t0 = time.time()
    cases = T.family_cases(L, "quadrants", range(2), 200) + T.family_cases(L, "sedov", range(2), 200)
    X, y, seen, npos = T.collect(L, cases, 40, 4, L.FP32_MIXED)
    t1 = time.time()
    ind, loss = T.train(L, X, y, epochs=15)
    t2 = time.time()
    tau = T.TAU_LO
    taus = (T.TAU_LO, T.TAU_HI)
    log(f"[bench] learned: {seen} cells seen, {npos} labelled troubled, {len(y)} training samples; collect "
        f"{t1 - t0:.1f} s, train {t2 - t1:.1f} s, tau_lo {tau:.3g}")
    out = {"training": {"families": "four-quadrant and near-vacuum blast, 2 seeds each, 200^2 lattices, 40 steps",
                        "cells_seen": seen, "positives": npos, "samples": int(len(y)), "final_loss": loss,
                        "collect_s": t1 - t0, "train_s": t2 - t1, "tau_lo": tau}}
    ms_p, kt_p, Qp, _ = time_steps(L, c3_mesh, c3_Q0, steps, warmup)
    ms_l, kt_l, Ql, cnt = time_steps(L, c3_mesh, c3_Q0, steps, warmup, ind, taus)
    n = c3_mesh.N
    out["tri_1M"] = {"plain_ms_per_step": ms_p, "learned_ms_per_step": ms_l, "learned_value": n / (ms_l * 1e-3),
                     "speedup_vs_plain_fp32": ms_p / ms_l, "rel_l1_learned_vs_plain": rel_l1(Ql, Qp),
                     "skip_fraction": cnt[0] / max(sum(cnt), 1),
                     "k_pre_us": {"plain": kt_p["k_pre"] * 1e3, "learned": kt_l["k_pre"] * 1e3},
                     "k_ind_us": kt_l["k_ind"] * 1e3}
    if fp64_Q is not None:
        out["tri_1M"]["rel_l1_learned_vs_fp64_plain"] = rel_l1(Ql, fp64_Q)
    log(f"[bench]   1M triangles: plain {ms_p:.3f} ms, learned {ms_l:.3f} ms per step; rel L1 learned vs plain "
        f"{out['tri_1M']['rel_l1_learned_vs_plain']:.2e}, skip {out['tri_1M']['skip_fraction']:.3f}")
    xy, tri, tags = I.ramp_channel(2_000_000, 0)
    Q0, inflow = I.ramp_state(xy, tri)
    mesh = L.Mesh.tri(xy, tri, I.ramp_bc(tags))
    kw = {"inflow": list(inflow)}
    ms_p, kt_p, Qp, _ = time_steps(L, mesh, Q0, steps, warmup, kw=kw)
    ms_l, kt_l, Ql, cnt = time_steps(L, mesh, Q0, steps, warmup, ind, taus, kw=kw)
    out["ramp_mach10"] = {"n_elem": mesh.N, "plain_ms_per_step": ms_p, "learned_ms_per_step": ms_l,
                          "plain_value": mesh.N / (ms_p * 1e-3), "learned_value": mesh.N / (ms_l * 1e-3),
                          "speedup_vs_plain_fp32": ms_p / ms_l, "rel_l1_learned_vs_plain": rel_l1(Ql, Qp),
                          "skip_fraction": cnt[0] / max(sum(cnt), 1),
                          "k_pre_us": {"plain": kt_p["k_pre"] * 1e3, "learned": kt_l["k_pre"] * 1e3},
                          "k_ind_us": kt_l["k_ind"] * 1e3}
    log(f"[bench]   ramp {mesh.N} triangles: plain {ms_p:.3f} ms, learned {ms_l:.3f} ms per step; rel L1 learned vs "
        f"plain {out['ramp_mach10']['rel_l1_learned_vs_plain']:.2e}, skip {out['ramp_mach10']['skip_fraction']:.3f}")
    return out, ind, taus


def diffraction_leg(L):
    """The paper's shock-diffraction problems (block step to t = 2.3, 120-degree wedge to t = 0.9)
    on unstructured meshes of the paper's size, and the block step on its 390 x 330 Cartesian mesh;
    whole runs through lxw_advance in both forms:
    steps, wall time, element-updates/s, and the density and pressure ranges against the paper's
    plots, with the shock-capturing limiter's relaxation factor 5 (500 lets spurious maxima grow on
    these domains; reported once per problem for comparison)."""
    import torch
    from paper_1601_08145_amd import inputs as I
    out = {}
    paper = {"step": {"rho": [0.066227, 7.0668], "p": [0.091, 37.0]}, "wedge": {"rho": [0.0665, 8.1], "p": [0.5, 118.0]}}
    for kind, n in (("step", 126018), ("wedge", 122046)):
        spec = I.DIFFRACTION[kind]
        xy, tri, tags = I.diffraction_domain(kind, n, 0)
        Q0, inflow = I.diffraction_state(xy, tri, kind)
        mesh = L.Mesh.tri(xy, tri, I.ramp_bc(tags))
        runs = []
        for prec, a0 in ((L.FP32_MIXED, 5.0), (L.FP64, 5.0), (L.FP32_MIXED, 500.0)):
            S = L.Solver(mesh, precision=prec, inflow=list(inflow), alpha0=a0)
            S.set_state(Q0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = S.advance(spec["t_end"])
            wall = time.perf_counter() - t0
            Q, t = S.get_state()
            rho = Q[:, 0, 0]
            p = 0.4 * (Q[:, 3, 0] - 0.5 * (Q[:, 1, 0] ** 2 + Q[:, 2, 0] ** 2) / rho)
            runs.append({"precision": "FP32_MIXED" if prec == L.FP32_MIXED else "FP64", "relaxation_factor": a0,
                         "steps": int(st.steps), "t": t, "wall_s": wall,
                         "element_updates_per_s": len(tri) * st.steps / wall,
                         "rho": [float(rho.min()), float(rho.max())], "p": [float(p.min()), float(p.max())]})
            log(f"[bench]   {kind} ({len(tri)} triangles), {runs[-1]['precision']}, factor {a0:g}: {st.steps} steps "
                f"to t = {t:g} in {wall:.2f} s ({runs[-1]['element_updates_per_s']:.3e} element-updates/s); "
                f"rho {rho.min():.4g}..{rho.max():.4g}, p {p.min():.4g}..{p.max():.4g}")
        out[kind] = {"n_elem": len(tri), "t_end": spec["t_end"], "mach": spec["mach"], "paper_plot_ranges": paper[kind],
                     "runs": runs}
    # the block step on the paper's 390 x 330 Cartesian mesh (Q2), the solid's cells removed
    nx, ny, box, bc, keep, Q0, inflow = I.diffraction_cart()
    mesh = L.Mesh.cart(nx, ny, *box, bc, keep=keep)
    runs = []
    for prec in (L.FP32_MIXED, L.FP64):
        S = L.Solver(mesh, precision=prec, inflow=list(inflow), alpha0=5.0)
        S.set_state(Q0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = S.advance(2.3)
        wall = time.perf_counter() - t0
        Q, t = S.get_state()
        rho = Q[:, 0, 0]
        p = 0.4 * (Q[:, 3, 0] - 0.5 * (Q[:, 1, 0] ** 2 + Q[:, 2, 0] ** 2) / rho)
        runs.append({"precision": "FP32_MIXED" if prec == L.FP32_MIXED else "FP64", "relaxation_factor": 5.0,
                     "steps": int(st.steps), "t": t, "wall_s": wall, "element_updates_per_s": len(Q0) * st.steps / wall,
                     "rho": [float(rho.min()), float(rho.max())], "p": [float(p.min()), float(p.max())]})
        log(f"[bench]   Cartesian step ({nx} x {ny}, {len(Q0)} cells), {runs[-1]['precision']}: {st.steps} steps to "
            f"t = {t:g} in {wall:.2f} s ({runs[-1]['element_updates_per_s']:.3e} element-updates/s); "
            f"rho {rho.min():.4g}..{rho.max():.4g}, p {p.min():.4g}..{p.max():.4g}")
    out["cartesian_step"] = {"nx": nx, "ny": ny, "n_elem": len(Q0), "t_end": 2.3, "mach": 5.09,
                             "paper_plot_ranges": paper["step"], "runs": runs}
    return out


def sedov_leg(L, t2=0.1):
    """The paper's Sedov blasts, whole runs through lxw_advance in both forms: 1D (dx = 1/100, to
    t = 0.001) and 2D on the disk of radius 1.1 with about 136,270 triangles (to t = t2, 0.1 by
    default; a later end time runs the FP32-mixed form only, with a progress line every 100k
    steps): steps,
    wall time, element-updates/s, the L1 density error against the similarity solution and the
    radius of the density maximum against the exact shock radius."""
    import torch
    from paper_1601_08145_amd import inputs as I
    from tests.exact_sedov import Sedov
    out = {}
    dx, T = 0.01, 1e-3
    n, x0, x1, Q0 = I.sedov_1d(dx)
    ex = Sedov(1, E=3.2e6)
    xc = x0 + (np.arange(n) + 0.5) * dx
    xs = xc[:, None] + ((np.arange(16) + 0.5) / 16 - 0.5)[None, :] * dx
    rho_e = ex.state(xs, T)[0].mean(axis=1)
    mesh = L.Mesh.line(n, x0, x1, L.BC_TRANSPARENT, L.BC_TRANSPARENT)
    runs = []
    for prec, exact in ((L.FP32_MIXED, 0), (L.FP64, 0), (L.FP64, 1)):
        S = L.Solver(mesh, precision=prec, cfl=0.1, theta_exact=exact)
        S.set_state(Q0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = S.advance(T)
        wall = time.perf_counter() - t0
        Q, t = S.get_state()
        l1 = float(np.abs(Q[:, 0, 0] - rho_e).sum() / np.abs(rho_e - 1.0).sum())
        runs.append({"precision": "FP32_MIXED" if prec == L.FP32_MIXED else "FP64", "theta_exact": exact,
                     "steps": int(st.steps), "t": t,
                     "wall_s": wall, "element_updates_per_s": n * st.steps / wall, "l1_rho_vs_similarity": l1,
                     "peak_x": float(abs(xc[np.argmax(Q[:, 0, 0])])), "rho_max": float(Q[:, 0, 0].max())})
        log(f"[bench]   Sedov 1D ({n} cells), {runs[-1]['precision']}{', exact factor' if exact else ''}: "
            f"{st.steps} steps in {wall:.2f} s; "
            f"L1(rho) vs similarity solution {l1:.4f}, peak at |x| = {runs[-1]['peak_x']:.3f} (exact shock {ex.radius(T):.3f})")
    out["1d"] = {"n_elem": n, "dx": dx, "t_end": T, "exact_shock_x": ex.radius(T), "runs": runs}
    xy, tri = I.sedov_disk()
    Q0 = I.sedov_disk_state(xy, tri)
    ex = Sedov(2, E=0.979264)
    a = xy[tri]
    w = np.array([[0.5, 0.5, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5],
                  [2 / 3, 1 / 6, 1 / 6], [1 / 6, 2 / 3, 1 / 6], [1 / 6, 1 / 6, 2 / 3]])
    pts = np.einsum("pk,nkd->npd", w, a)
    T2 = t2
    rho_e = ex.state(np.hypot(pts[..., 0], pts[..., 1]), T2)[0].mean(axis=1)
    area = 0.5 * np.abs((a[:, 1, 0] - a[:, 0, 0]) * (a[:, 2, 1] - a[:, 0, 1]) - (a[:, 1, 1] - a[:, 0, 1]) * (a[:, 2, 0] - a[:, 0, 0]))
    r = np.hypot(a.mean(axis=1)[:, 0], a.mean(axis=1)[:, 1])
    mesh = L.Mesh.tri(xy, tri)
    runs = []
    forms = ((L.FP32_MIXED, 0), (L.FP64, 0), (L.FP32_MIXED, 1)) if T2 <= 0.1 else ((L.FP32_MIXED, 0),)
    for prec, exact in forms:
        S = L.Solver(mesh, precision=prec, theta_exact=exact)
        S.set_state(Q0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps, t = 0, 0.0
        while t < T2:
            st = S.advance(T2, 100000)
            steps += st.steps
            t = st.t
            if t < T2:
                log(f"[bench]     t = {t:.4f} after {steps} steps, last dt {st.last_dt:.3e}, "
                    f"{time.perf_counter() - t0:.0f} s")
        st.steps = steps
        wall = time.perf_counter() - t0
        Q, t = S.get_state()
        rho = Q[:, 0, 0]
        l1 = float(np.sum(np.abs(rho - rho_e) * area) / np.sum(np.abs(rho_e - 1.0) * area))
        runs.append({"precision": "FP32_MIXED" if prec == L.FP32_MIXED else "FP64", "theta_exact": exact,
                     "steps": int(st.steps), "t": t,
                     "wall_s": wall, "element_updates_per_s": len(tri) * st.steps / wall, "l1_rho_vs_similarity": l1,
                     "peak_r": float(r[np.argmax(rho)]), "rho_max": float(rho.max())})
        log(f"[bench]   Sedov 2D ({len(tri)} triangles), {runs[-1]['precision']}{', exact factor' if exact else ''}: "
            f"{st.steps} steps in {wall:.2f} s "
            f"({runs[-1]['element_updates_per_s']:.3e} element-updates/s); L1(rho) vs similarity solution {l1:.4f}, "
            f"peak {rho.max():.3f} at r = {runs[-1]['peak_r']:.4f} (exact shock {ex.radius(T2):.4f})")
    out["2d_disk"] = {"n_elem": len(tri), "t_end": T2, "exact_shock_r": ex.radius(T2), "runs": runs}
    # to the usual end time t = 1 with the wave speed from the cell averages only
    rho_e = ex.state(np.hypot(pts[..., 0], pts[..., 1]), 1.0)[0].mean(axis=1)
    S = L.Solver(mesh, precision=L.FP32_MIXED, wave_speed=L.SPEED_AVERAGES)
    S.set_state(Q0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps, t = 0, 0.0
    while t < 1.0:
        st = S.advance(1.0, 50000)
        steps += st.steps
        t = st.t
        log(f"[bench]     t = {t:.4f} after {steps} steps, {time.perf_counter() - t0:.0f} s")
    wall = time.perf_counter() - t0
    Q, t = S.get_state()
    rho = Q[:, 0, 0]
    l1 = float(np.sum(np.abs(rho - rho_e) * area) / np.sum(np.abs(rho_e - 1.0) * area))
    out["2d_disk_t1_average_speeds"] = {"precision": "FP32_MIXED", "wave_speed": "cell averages", "t_end": 1.0,
                                        "steps": steps, "wall_s": wall,
                                        "element_updates_per_s": len(tri) * steps / wall,
                                        "l1_rho_vs_similarity": l1, "peak_r": float(r[np.argmax(rho)]),
                                        "rho_max": float(rho.max()), "exact_shock_r": ex.radius(1.0)}
    log(f"[bench]   Sedov 2D to t = 1, wave speed from the cell averages: {steps} steps in {wall:.1f} s; "
        f"L1(rho) vs similarity solution {l1:.4f}, peak {rho.max():.3f} at r = {r[np.argmax(rho)]:.4f} "
        f"(exact shock {ex.radius(1.0):.4f})")
    return out


def cartesian_blast_leg(L, n=512, steps=100, warmup=5):
    """The Cartesian Q2 workload: a near-vacuum blast (rho = 1, u = 0, p = 1e-10, energy 0.98 in
    the four centre cells) on a periodic n x n mesh of [-1, 1]^2, both forms: ms per step from
    graph replay after `warmup` steps, per-kernel times from HIP events, and the FP32-mixed form's
    relative L1 difference to FP64 after the same steps."""
    from paper_1601_08145_amd import inputs as I
    mesh = L.Mesh.cart(n, n, -1, 1, -1, 1, [0, 0, 0, 0])
    Q0 = I.sedov_cart_state(n, n)
    out = {"n_elem": n * n, "steps": steps}
    res = {}
    for prec, name in ((L.FP32_MIXED, "FP32_MIXED"), (L.FP64, "FP64")):
        r = time_gpu(L, mesh, Q0, prec, steps, warmup)
        res[name] = r
        rho = r["Q"][:, 0, 0]
        out[name] = {"ms_per_step": r["ms_graph"] / steps, "element_updates_per_s": n * n * steps / (r["ms_graph"] * 1e-3),
                     "kernels_ms": {k: v[0] / max(v[1], 1) for k, v in r["kernels"].items() if v[1]},
                     "rho_min": float(rho.min()), "t": r["t"]}
        log(f"[bench]   Cartesian blast {n}^2, {name}: {r['ms_graph'] / steps:.3f} ms/step "
            f"({out[name]['element_updates_per_s']:.3e} element-updates/s); kernels "
            f"{ {k: round(v * 1e3, 1) for k, v in out[name]['kernels_ms'].items()} } us")
    out["rel_l1_fp32_vs_fp64"] = rel_l1(res["FP32_MIXED"]["Q"], res["FP64"]["Q"])
    log(f"[bench]   FP32-mixed vs FP64 after {warmup + 2 * steps} steps: rel L1 {out['rel_l1_fp32_vs_fp64']:.2e}")
    return out


def p3_leg(L, mesh, xy, tri, steps, warmup):
    """The degree-3 step (P3, F_T to dt^3) on the benchmark's triangle mesh and four-quadrant data
    (averages, higher modes zero), CFL 0.05, both forms: ms per step from graph replay, per-kernel
    times, element and degree-of-freedom updates per second, and FP32-mixed vs FP64 after the same
    steps."""
    from paper_1601_08145_amd import inputs as I
    Q0 = I.averages_to_modal(I.cell_average_state(I.four_quadrant_fn(0), I.tri_sample_points(xy, tri, 2), 1.4), 10)
    n = mesh.N
    out = {"n_elem": n, "modes": 10, "cfl": 0.05, "steps": steps}
    res = {}
    for prec, name in ((L.FP32_MIXED, "FP32_MIXED"), (L.FP64, "FP64")):
        r = time_gpu(L, mesh, Q0, prec, steps, warmup, kw={"degree": 3, "cfl": 0.05})
        res[name] = r
        ms = r["ms_graph"] / steps
        out[name] = {"ms_per_step": ms, "element_updates_per_s": n / (ms * 1e-3), "dof_updates_per_s": 10 * n / (ms * 1e-3),
                     "kernels_ms": {k: v[0] / max(v[1], 1) for k, v in r["kernels"].items() if v[1]}}
        log(f"[bench]   P3 triangles, {name}: {ms:.3f} ms/step ({out[name]['element_updates_per_s']:.3e} element-updates/s, "
            f"{out[name]['dof_updates_per_s']:.3e} modes/s); kernels "
            f"{ {k: round(v * 1e3, 1) for k, v in out[name]['kernels_ms'].items()} } us")
    out["rel_l1_fp32_vs_fp64"] = rel_l1(res["FP32_MIXED"]["Q"], res["FP64"]["Q"])
    log(f"[bench]   P3 FP32-mixed vs FP64 after {warmup + 2 * steps} steps: rel L1 {out['rel_l1_fp32_vs_fp64']:.2e}")
    return out


def tet_leg(L, steps, warmup, n=56):
    """The step on tetrahedra (3D P2): a periodic jittered (n-1)^3-cube lattice split into six
    tetrahedra per cube (998,250 at n = 56), the plane density wave along (1, 1, 1) with a uniform
    flow, both forms: ms per step from graph replay, per-kernel times, element-updates per second,
    FP32-mixed vs FP64 after the same steps."""
    from paper_1601_08145_amd import inputs as I
    xyz, tet = I.lattice_tets(n, 3, periodic=True)
    tags = I.boundary_tags_tet(xyz, tet, (0, 1, 0, 1, 0, 1), [0] * 6)
    mesh = L.Mesh.tet(xyz, tet, tags, (1.0, 1.0, 1.0))
    xq = mesh.quad_points()
    kv, u0 = np.array([1.0, 1.0, 1.0]), np.array([0.6, -0.3, 0.4])
    rho = 1 + 0.3 * np.sin(2 * np.pi * (xq @ kv))
    one = np.ones_like(rho)
    prim = np.stack([rho, u0[0] * one, u0[1] * one, u0[2] * one, one], -1)
    cons = np.concatenate([prim[..., :1], prim[..., :1] * prim[..., 1:4],
                           prim[..., 4:] / 0.4 + 0.5 * prim[..., :1] * np.sum(prim[..., 1:4] ** 2, -1, keepdims=True)], -1)
    Q0 = mesh.project(cons)
    N = mesh.N
    out = {"n_elem": N, "modes": 10, "workload": "plane density wave, periodic jittered tetrahedra", "steps": steps}
    res = {}
    for prec, name in ((L.FP32_MIXED, "FP32_MIXED"), (L.FP64, "FP64")):
        r = time_gpu(L, mesh, Q0, prec, steps, warmup)
        res[name] = r
        ms = r["ms_graph"] / steps
        out[name] = {"ms_per_step": ms, "element_updates_per_s": N / (ms * 1e-3),
                     "kernels_ms": {k: v[0] / max(v[1], 1) for k, v in r["kernels"].items() if v[1]}}
        log(f"[bench]   tetrahedra {N}, {name}: {ms:.3f} ms/step ({out[name]['element_updates_per_s']:.3e} element-updates/s); "
            f"kernels { {k: round(v * 1e3, 1) for k, v in out[name]['kernels_ms'].items()} } us")
    out["rel_l1_fp32_vs_fp64"] = rel_l1(res["FP32_MIXED"]["Q"], res["FP64"]["Q"])
    log(f"[bench]   tetrahedra FP32-mixed vs FP64 after {warmup + 2 * steps} steps: rel L1 {out['rel_l1_fp32_vs_fp64']:.2e}")
    return out


def sedov_disk_steps(L, steps, warmup, t_start=0.05):
    """The 2D Sedov blast (136k triangles, FP32-mixed), advanced to t_start, then `warmup` and
    `steps` steps replayed from the graph: the near-vacuum core keeps the flux and moment limiters
    busy."""
    from paper_1601_08145_amd import inputs as I
    xy, tri = I.sedov_disk()
    S = L.Solver(L.Mesh.tri(xy, tri), precision=L.FP32_MIXED)
    S.set_state(I.sedov_disk_state(xy, tri))
    st = S.advance(t_start)
    S.run_steps(warmup)
    S.sync()
    ms = _timed(S, steps)
    log(f"[bench] Sedov disk ({len(tri)} triangles) from t = {t_start} ({st.steps} steps): "
        f"{ms / steps:.4f} ms/step over {steps} steps")
    return {"n_elem": len(tri), "t_start": t_start, "steps_to_start": int(st.steps), "ms_per_step": ms / steps}


def equal_l1_leg(L, ind, taus, sizes=(48, 96, 192), T=1.0):
    """Each form on an exact solution (Shu's isentropic vortex advected by (1, 1) on a periodic
    [-5,5]^2 Delaunay mesh), to time T, at three resolutions: L1 error of the cell averages against
    the exact ones (both from the library's 7-point projection).  Where the discretisation error is
    far above float32 rounding the forms agree; on fine meshes float32 rounding sets a floor."""
    from paper_1601_08145_amd import inputs as I
    out = {"workload": f"isentropic vortex (strength 5) advected by (1,1) to t = {T}, periodic [-5,5]^2, "
                       f"jittered-lattice Delaunay meshes, CFL 0.08", "T": T, "meshes": []}
    for n in sizes:
        xy, tri = I.lattice_delaunay(n, 5, box=(-5.0, 5.0, -5.0, 5.0), periodic=True)
        tags = I.boundary_tags(xy, tri, (-5.0, 5.0, -5.0, 5.0), [0, 0, 0, 0])
        mesh = L.Mesh.tri(xy, tri, tags, (10.0, 10.0))
        pts = mesh.quad_points()
        Q0 = mesh.project(I.prim_to_cons(I.vortex_fn(0.0)(pts), 1.4))
        ex = mesh.project(I.prim_to_cons(I.vortex_fn(T)(pts), 1.4))[:, :, 0]
        a = xy[tri]
        area = 0.5 * np.abs((a[:, 1, 0] - a[:, 0, 0]) * (a[:, 2, 1] - a[:, 0, 1])
                            - (a[:, 1, 1] - a[:, 0, 1]) * (a[:, 2, 0] - a[:, 0, 0]))
        row = {"n_elem": mesh.N, "forms": {}}
        for name, prec, use_ind in (("fp64_plain", L.FP64, False), ("fp32_mixed", L.FP32_MIXED, False),
                                    ("fp32_mixed_learned", L.FP32_MIXED, True)):
            if use_ind and ind is None:
                continue
            S = L.Solver(mesh, precision=prec)
            S.set_state(Q0)
            if use_ind:
                S.set_indicator(ind, *taus)
            st = S.advance(T)
            Q, _ = S.get_state()
            err = float(np.sum(np.abs(Q[:, 0, 0] - ex[:, 0]) * area) / np.sum(area))
            row["forms"][name] = {"l1_rho": err, "steps": st.steps}
        f = row["forms"]
        row["fp32_over_fp64_l1"] = f["fp32_mixed"]["l1_rho"] / f["fp64_plain"]["l1_rho"]
        log(f"[bench]   vortex {mesh.N} triangles: L1(rho) fp64 {f['fp64_plain']['l1_rho']:.4e}, fp32 "
            f"{f['fp32_mixed']['l1_rho']:.4e}" + (f", learned {f['fp32_mixed_learned']['l1_rho']:.4e}"
                                                  if "fp32_mixed_learned" in f else ""))
        out["meshes"].append(row)
    out["sedov_disk"] = equal_l1_sedov(L, ind, taus)
    return out


def equal_l1_sedov(L, ind, taus, T=0.1):
    """Each form on the 2D Sedov blast (136k-triangle disk, to t = T), where the shock-capturing
    limiter acts every step and the similarity solution is exact: L1 density error against it
    (relative to the blast's density deviation) and the whole run's time per step."""
    import torch
    from paper_1601_08145_amd import inputs as I
    from tests.exact_sedov import Sedov
    xy, tri = I.sedov_disk()
    Q0 = I.sedov_disk_state(xy, tri)
    a = xy[tri]
    w = np.array([[0.5, 0.5, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5],
                  [2 / 3, 1 / 6, 1 / 6], [1 / 6, 2 / 3, 1 / 6], [1 / 6, 1 / 6, 2 / 3]])
    pts = np.einsum("pk,nkd->npd", w, a)
    rho_e = Sedov(2, E=0.979264).state(np.hypot(pts[..., 0], pts[..., 1]), T)[0].mean(axis=1)
    area = 0.5 * np.abs((a[:, 1, 0] - a[:, 0, 0]) * (a[:, 2, 1] - a[:, 0, 1]) - (a[:, 1, 1] - a[:, 0, 1]) * (a[:, 2, 0] - a[:, 0, 0]))
    mesh = L.Mesh.tri(xy, tri)
    out = {"workload": f"2D Sedov blast on the {len(tri)}-triangle disk to t = {T}, L1 of rho against the "
                       "similarity solution over that of its deviation from the background", "forms": {}}
    for name, prec, use_ind in (("fp64_plain", L.FP64, False), ("fp32_mixed", L.FP32_MIXED, False),
                                ("fp32_mixed_learned", L.FP32_MIXED, True)):
        if use_ind and ind is None:
            continue
        S = L.Solver(mesh, precision=prec)
        S.set_state(Q0)
        if use_ind:
            S.set_indicator(ind, *taus)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = S.advance(T)
        wall = time.perf_counter() - t0
        Q, _ = S.get_state()
        l1 = float(np.sum(np.abs(Q[:, 0, 0] - rho_e) * area) / np.sum(np.abs(rho_e - 1.0) * area))
        f = {"l1_rho_vs_similarity": l1, "steps": int(st.steps), "ms_per_step": wall / st.steps * 1e3}
        if use_ind:
            cnt = S.indicator_decisions(False)[0].tolist()
            f["skip_fraction"] = cnt[0] / max(sum(cnt), 1)
        out["forms"][name] = f
        log(f"[bench]   Sedov disk {name}: L1(rho) vs similarity {l1:.4f}, {st.steps} steps, "
            f"{f['ms_per_step']:.4f} ms/step")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-kernel-events", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-mesh batched leg")
    ap.add_argument("--batched-only", action="store_true", help="run only the batched leg (for profiling)")
    ap.add_argument("--sedov-disk-only", action="store_true",
                    help="only steps of the 2D Sedov blast mid-run (near-vacuum limiting; for profiling)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-indicator leg")
    ap.add_argument("--learned-only", action="store_true", help="run only the learned-indicator leg (for profiling)")
    ap.add_argument("--no-equal-l1", action="store_true", help="skip the equal-L1 comparison on the vortex")
    ap.add_argument("--no-diffraction", action="store_true", help="skip the shock-diffraction runs")
    ap.add_argument("--no-sedov", action="store_true", help="skip the Sedov blast runs")
    ap.add_argument("--sedov-2d-end", type=float, default=0.1, help="end time of the 2D Sedov run (default 0.1)")
    ap.add_argument("--no-exact-theta", action="store_true", help="skip the exact moment-limiter factor leg")
    ap.add_argument("--no-cartesian", action="store_true", help="skip the Cartesian Q2 blast leg")
    ap.add_argument("--no-p3", action="store_true", help="skip the degree-3 leg")
    ap.add_argument("--no-tet", action="store_true", help="skip the tetrahedra (3D) leg")
    ap.add_argument("--tet-only", action="store_true", help="run only the tetrahedra leg (for profiling)")
    ap.add_argument("--p3-only", action="store_true", help="run only the degree-3 leg (for profiling)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only copy a float32 buffer of BYTES bytes 3 times (reference for HBM counters)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        n = args.copy_probe // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        ms = []
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            b.copy_(a)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        # bytes read + written per copy over the fastest of the three
        print(json.dumps({"copy_probe_bytes": n * 4, "copies": 3, "ms": ms,
                          "GBs_read_plus_write": 2 * n * 4 / (min(ms) * 1e-3) / 1e9}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the LxW-DG step here is a "
                          "single-GPU build (multi-GPU sharding is a design note, not implemented)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_1601_08145_amd import lxw as L

    if args.batched_only:
        print(json.dumps({"batched": batched_leg(L, args.steps, args.warmup)}), flush=True)
        return
    if args.tet_only:
        print(json.dumps({"tet": tet_leg(L, args.steps, args.warmup)}), flush=True)
        return
    if args.sedov_disk_only:
        print(json.dumps({"sedov_disk": sedov_disk_steps(L, args.steps, args.warmup)}), flush=True)
        return

    xy, tri, Q0 = build_workload()
    mesh = L.Mesh.tri(xy, tri)
    N = mesh.N
    if args.p3_only:
        print(json.dumps({"p3": p3_leg(L, mesh, xy, tri, args.steps, args.warmup)}), flush=True)
        return
    if args.learned_only:
        print(json.dumps({"learned": learned_leg(L, args.steps, args.warmup, mesh, Q0)[0]}), flush=True)
        return

    log(f"[bench] FP32-mixed: {args.warmup} warm-up + 2 x {args.steps} timed steps")
    mix = time_gpu(L, mesh, Q0, L.FP32_MIXED, args.steps, args.warmup, not args.no_kernel_events)
    # the headline is the library's default path (lxw_run_steps replays the captured step); the
    # per-kernel durations come from the region of equal length just before it
    ms_step = mix["ms_graph"] / args.steps
    value = N * args.steps / (mix["ms_graph"] * 1e-3)
    log(f"[bench]   {ms_step:.3f} ms/step (graph replay), {value:.4e} element-updates/s; with per-kernel "
        f"events {mix['ms_total'] / args.steps:.3f} ms/step")

    out = {"metric": METRIC, "value": value, "unit": "element-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32 (f64 cell averages and flux limiter)", "data": "synthetic",
           "config": {"workload": "2D Euler, P2 triangles, 999,698-triangle Delaunay mesh of a 708^2 lattice "
                                  "jittered 0.3h on [0,1]^2, four-quadrant Riemann data seed 0, transparent "
                                  "boundaries, CFL 0.08, plain shock limiter",
                      "n_elem": N, "n_edge": mesh.E, "precision": "FP32_MIXED"},
           "timing": {"value_region": "steps replayed from the captured HIP graph (the library default)",
                      "kernel_events_region": {"ms_per_step": mix["ms_total"] / args.steps,
                                               "note": "the same number of steps just before, every kernel "
                                                       "launched with HIP events around it; per-kernel "
                                                       "durations and the roofline come from it"}}}

    if mix["kernels"]:
        kt = {k: {"ms_avg": v[0] / max(v[1], 1), "launches": v[1]} for k, v in mix["kernels"].items()}
        out["kernels"] = kt
        out["roofline"] = kelem_roofline(kt["k_elem"]["ms_avg"], N, traffic_ok=True, ms_per_step=ms_step)

    cr = copy_rate()
    out["hbm_copy_probe"] = {"GBs": cr / 1e9, "frac_of_peak": cr / 1e9 / PEAK_HBM_GBS,
                             "note": "device copy of 1 GiB, bytes read + written, fastest of 5"}
    log(f"[bench] 1 GiB device copy: {cr / 1e12:.2f} TB/s read + write")
    if mix["kernels"] and traffic_valid():
        # measured HBM bytes per launch over this run's per-kernel times
        hk = {}
        for k, b in TRAFFIC["bytes_per_launch"].items():
            gbs = b / (out["kernels"][k]["ms_avg"] * 1e-3) / 1e9
            hk[k] = {"traffic_bytes": b, "achieved_GBs": gbs, "frac_of_peak": gbs / PEAK_HBM_GBS,
                     "frac_of_copy_probe": gbs / (cr / 1e9)}
        out["hbm_kernels"] = hk

    if not args.no_fp64:
        log(f"[bench] FP64 plain: {args.warmup} warm-up + {args.steps} timed steps")
        f64 = time_gpu(L, mesh, Q0, L.FP64, args.steps, args.warmup, not args.no_kernel_events)
        v64 = N * args.steps / (f64["ms_graph"] * 1e-3)
        a, b = mix["Q"], f64["Q"]
        rel = max(float(np.abs(a[:, v] - b[:, v]).sum() / np.abs(b[:, v]).sum()) for v in range(4))
        out["fp64_plain"] = {"value": v64, "ms_per_step": f64["ms_graph"] / args.steps,
                             "kernel_events_ms_per_step": f64["ms_total"] / args.steps,
                             "kernels": {k: {"ms_avg": v[0] / max(v[1], 1), "launches": v[1]}
                                         for k, v in f64["kernels"].items()}}
        out["mixed_vs_fp64"] = {"speedup": value / v64, "rel_l1_state_diff": rel,
                                "note": f"states after {args.warmup + 2 * args.steps} steps from the same input"}
        log(f"[bench]   FP64 {v64:.4e} element-updates/s; mixed/FP64 {value / v64:.2f}x; rel L1 diff {rel:.2e}")

    if not args.no_exact_theta:
        # the moment limiter with the exact pressure factor, on the same workload
        ms_p, kt_p, Qp, _ = time_steps(L, mesh, Q0, args.steps, args.warmup)
        ms_e, kt_e, Qe, _ = time_steps(L, mesh, Q0, args.steps, args.warmup, kw={"theta_exact": 1})
        out["exact_theta"] = {"ms_per_step": ms_e, "plain_ms_per_step": ms_p, "k_pre_ms": kt_e.get("k_pre"),
                              "plain_k_pre_ms": kt_p.get("k_pre"), "rel_l1_vs_plain": rel_l1(Qe, Qp),
                              "note": f"FP32-mixed, states after {args.warmup + 2 * args.steps} steps"}
        log(f"[bench] exact moment-limiter factor: {ms_e:.3f} ms/step (plain {ms_p:.3f}), k_pre "
            f"{kt_e.get('k_pre', 0) * 1e3:.1f} us (plain {kt_p.get('k_pre', 0) * 1e3:.1f}); rel L1 vs plain "
            f"{out['exact_theta']['rel_l1_vs_plain']:.2e}")

    if not args.no_batched:
        out["batched"] = batched_leg(L, args.steps, args.warmup)

    ind, taus = None, None
    if not args.no_learned:
        out["learned"], ind, taus = learned_leg(L, args.steps, args.warmup, mesh, Q0,
                                                f64["Q"] if not args.no_fp64 else None)
    if not args.no_diffraction:
        log("[bench] shock diffraction (whole runs)")
        out["diffraction"] = diffraction_leg(L)
    if not args.no_p3:
        log("[bench] degree 3 (P3 triangles)")
        out["p3"] = p3_leg(L, mesh, xy, tri, args.steps, args.warmup)
    if not args.no_tet:
        log("[bench] tetrahedra (3D)")
        out["tet"] = tet_leg(L, args.steps, args.warmup)
    if not args.no_cartesian:
        log("[bench] Cartesian Q2 near-vacuum blast")
        out["cartesian_blast"] = cartesian_blast_leg(L)
    if not args.no_sedov:
        log("[bench] Sedov blasts (whole runs)")
        out["sedov"] = sedov_leg(L, args.sedov_2d_end)
    if not args.no_equal_l1:
        log("[bench] equal-L1 comparison on an exact solution")
        out["equal_l1"] = equal_l1_leg(L, ind, taus)

    if not args.no_cpu_baseline:
        log("[bench] CPU baseline (oracle, about 10 s of steps)")
        out["cpu_baseline"] = cpu_baseline(xy, tri, Q0)
        cb = out["cpu_baseline"]
        log(f"[bench]   {cb['value']:.4e} element-updates/s on {cb['cores']} threads, {cb['one_thread']['value']:.4e} on 1 "
            f"({cb['cpu_model']})")

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
