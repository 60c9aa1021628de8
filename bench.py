"""Benchmark: batched implicit neutrino-matter coupling solves on one MI355X.

Workload: the synthetic supernova-like radial profile, 2^16 spatial points,
3 species (nu_e, anti-nu_e, nu_x), 32 energy nodes (16 geometric elements x 2
Legendre-Gauss nodes on 1-300 MeV), full physics (emission/absorption,
isoenergetic scattering, NES and pair kernels), FP64, Anderson memory 3,
tolerance 1e-10.  One bench step = one replay of a captured HIP graph that
restores the initial state and runs 10 chained implicit steps (each the
persistent work-queue kernel over all points, output feeding the next step).

Metric: implicit point-solves per second (points below 1e7 g/cm^3, where the
coupling is switched off and the state passes through, are not counted).
The JSON line also carries the roofline of the solve kernel (FP64 vector ALU
bound; algorithmic FLOPs per launch / kernel time from HIP events captured
around each launch in the graph) and the CPU oracle timed on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

NS = 3
STEPS_PER_GRAPH = 10
# name: (energy elements, points, workload id of the draws, traffic tag, kernel label)
WORKLOADS = {
    "profile32": (16, 1 << 16, 3, "fwd_pair_kernel_nq32_ns3",
                  "fwd_pair_kernel<3> (persistent point solve, two points per wavefront)"),
    "profile64": (32, 1 << 18, 4, "fwd64_kernel_nq64_ns3", "fwd64_kernel<3> (persistent point solve, 64 nodes)"),
}
NQ, P_POINTS = 32, 1 << 16  # headline workload
PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector, published
PEAK_HBM_GBS = 8000.0


def flops_per_point(n_inner, n_outer, nq=32, ns=NS):
    """Algorithmic FLOPs of one point-solve (FMA = 2): per inner iteration the
    four energy-coupling mat-vecs of every species (8 ns nq^2) and pointwise
    plus Anderson work (40 ns nq); per outer iteration the kernel build and
    matter update (4 nq^2 + 30 ns nq)."""
    return n_inner * (8 * ns * nq * nq + 40 * ns * nq) + n_outer * (4 * nq * nq + 30 * ns * nq)


def flops_per_point_v(n_inner, n_outer, nq=32, ns=NS):
    """Algorithmic FLOPs of one O(v) point-solve (FMA = 2), counted from the
    two-points-per-wavefront kernel: per inner iteration the four
    energy-coupling mat-vecs of every species (8 ns nq^2) and, per species and
    node, the Minerbo closure with the velocity products (47), the right-hand
    sides and quotients of the four moments (41), the Anderson step over them
    (72) and the convergence sums (14), together 174 ns nq; per outer
    iteration the kernel build (4 nq^2), the opacities and equilibrium (30 ns
    nq) and the Eulerian integrals with their closure (70 ns nq)."""
    return n_inner * (8 * ns * nq * nq + 174 * ns * nq) + n_outer * (4 * nq * nq + 100 * ns * nq)


def flops_per_point_v_phi1(n_inner, n_outer, nq=32, ns=NS):
    """Algorithmic FLOPs of one O(v) point-solve with the linear-order Phi_1
    corrections (FMA = 2): the O(v) count plus, per inner iteration, the four
    Phi_1 contractions of every species against each of the three flux
    components (24 ns nq^2) and, per species and node, the two combinations
    of the contracted vectors per component (18) and the Phi_1 collision terms
    of the closure (52), together 70 ns nq."""
    return flops_per_point_v(n_inner, n_outer, nq, ns) + n_inner * (24 * ns * nq * nq + 70 * ns * nq)


def flops_per_node_c2p(iters):
    """Algorithmic FLOPs of one primitive-moment recovery (FMA = 2), per
    iteration of the fixed-point map: the Minerbo closure with the velocity
    products (47), the relaxed map (16) and residual (4), the Anderson step
    over the 4-vector (79: differences, Gram sums, the 2 x 2 solve, mixing)
    and the convergence test (12), together 158; per node the scaling, the
    step parameter and the reference norm (30)."""
    return 158 * iters + 30


def bytes_per_node_c2p(ns=NS, nq=32):
    """Algorithmic HBM bytes of one node recovery: read N and G (4 doubles),
    write D and I (4 doubles) and the iteration count (int32), plus the
    point's velocity (3 doubles) shared by its ns * nq nodes."""
    return 4 * 8 + 4 * 8 + 4 + 3 * 8 / (ns * nq)


def bytes_per_point(nq=32, ns=NS):
    """Algorithmic HBM bytes of one point-solve: read D*, I* and 3 scalars
    (rho11, Ye*, e*), write D, I, 3 scalars (Ye, e, T) and 3 int32 counters."""
    return 2 * ns * nq * 8 + 3 * 8 + 2 * ns * nq * 8 + 3 * 8 + 3 * 4


def bytes_per_point_v(nq=32, ns=NS):
    """Algorithmic HBM bytes of one O(v) point-solve: read D*, the three flux
    components and 6 scalars (rho11, Ye*, ef*, v*), write D, I, 6 scalars
    (Ye, ef, v, T) and 3 int32 counters."""
    return 2 * 4 * ns * nq * 8 + 6 * 8 + 6 * 8 + 3 * 4


# O(v) workload: the inner loop is solved 100 times tighter than the outer one
# (its lambda < 1 fixed-point map converges linearly, and the residual error,
# amplified by the neutrino/matter reservoir ratio at the low-density edge of
# the profile, would otherwise exceed the outer tolerance there)
V_TOL_INNER, V_TOL_OUTER = 1e-12, 1e-10
V_WID = 6
# linear-order corrections of the Phi_1 workload: Phi_1 = r Phi_0 per process
PHI1_NES, PHI1_PAIR = 0.3, -0.25


def cpu_baseline_v(steps: int, threads: int, mode: str = "solve"):
    """The oracle's O(v) solve (mode "solve"), the same with the Phi_1
    corrections ("phi1") or its PD-ARS step ("pdars") on the moving profile:
    all 2^16 points, `steps` chained steps from the initial state."""
    import numpy as np

    import oracle as O
    from paper_2601_00976_amd import solver as S
    from paper_2601_00976_amd import workloads as W

    O.build(force=False)
    d = W.radial_profile_v(P=P_POINTS, wid=V_WID)
    m = O.Model(n_elem=16, overrides=dict(phi1_nes=PHI1_NES, phi1_pair=PHI1_PAIR) if mode == "phi1" else {})
    theta = m.default_theta(S.DEFAULT_A_NES, S.DEFAULT_A_PAIR)
    D, _, e0 = m.init_state(d.T, d.rho11, d.ye, d.uD, d.uI)
    I = 0.1 * D[:, :, None, :] * d.uI3
    ef = e0 + 0.5 * O.MU_C2 * np.sum(d.v * d.v, axis=1)
    ye, v = d.ye.copy(), d.v.copy()
    prm = O.Params(tol_inner=V_TOL_INNER, tol_outer=V_TOL_OUTER)
    solved = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        if mode == "pdars":
            r = O.pdars_step_v(m, prm, theta, W.DTAU_KM, D, I, d.rho11, ye, ef, v, nthreads=threads)
        else:
            r = O.solve_batch_v(m, prm, theta, W.DTAU_KM, D, I, d.rho11, ye, ef, v, nthreads=threads)
        D, I, ye, ef, v = r["D"], r["I"], r["ye"], r["ef"], r["v"]
        solved += int(np.sum(r["n_outer"] > 0))
    dt = time.perf_counter() - t0
    unit = "point-steps/s" if mode == "pdars" else "point-solves/s"
    return dict(value=solved / dt, unit=unit, cores=threads, kind="oracle",
                sample=f"all {P_POINTS} moving-profile points, {steps} chained steps, {solved} solved point-steps "
                       f"in {dt:.1f} s")


def cpu_baseline_c2p(threads: int, min_seconds: float = 10.0):
    """The oracle's primitive-moment recovery of the same conserved moments
    (every node of the profile), repeated until `min_seconds` have passed."""
    import numpy as np

    import oracle as O
    from paper_2601_00976_amd import workloads as W

    O.build(force=False)
    d = W.radial_profile_v(P=P_POINTS, wid=V_WID)
    m = O.Model(n_elem=16)
    D, _, _ = m.init_state(d.T, d.rho11, d.ye, d.uD, d.uI)
    I = 0.1 * D[:, :, None, :] * d.uI3
    N, G, v = D, np.ascontiguousarray(I), np.ascontiguousarray(d.v)
    done, reps = 0, 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < min_seconds:
        _, _, it = O.primitive_batch(m, N, G, v, nthreads=threads)
        done += it.size
        reps += 1
    dt = time.perf_counter() - t0
    return dict(value=done / dt, unit="node-recoveries/s", cores=threads, kind="oracle",
                sample=f"every node of the moving profile ({it.size}) x {reps}: {done} recoveries in {dt:.1f} s")


def run_velocity(args, mode: str = "solve"):
    """The O(v) solve (nonzero fluid velocity) on the moving radial profile:
    2^16 points, 3 species, 32 nodes, 10 chained in-place steps per captured
    graph, timed and accounted as the static workload.  mode "phi1": the same
    solve with the linear-order Phi_1 corrections (Phi_1 = r Phi_0, r = 0.3
    for NES and -0.25 for pair); mode "pdars": each step is one PD-ARS IMEX
    step of the coupling (two solves, dt and dt / 2, with the primitive
    recovery between them)."""
    import numpy as np
    import torch

    from paper_2601_00976_amd import autotune as AT
    from paper_2601_00976_amd import solver as S
    from paper_2601_00976_amd import workloads as W

    dev = torch.device("cuda:0")
    model = S.Model(S.Grid(16), **(dict(phi1_nes=PHI1_NES, phi1_pair=PHI1_PAIR) if mode == "phi1" else {}))
    params = S.Params(tol_inner=V_TOL_INNER, tol_outer=V_TOL_OUTER)
    t = S.to_device(W.radial_profile_v(P=P_POINTS, wid=V_WID), dev)
    D0, I0, ef0 = S.init_state_v(model, t)
    theta = model.default_theta()
    launch = S.LaunchConfig(chunk=args.chunk or 1, blocks_per_cu=args.blocks_per_cu or 0)
    if mode == "phi1" and args.kernel_store == "wave":
        launch.kernel_store = 5
        kernel_label, traffic_tag = ("fwd_v_kernel<3, true, true> (persistent O(v) point solve with the Phi_1 "
                                     "corrections, one point per wavefront)"), "fwd_v_kernel_nq32_ns3_phi1"
    elif mode == "phi1":
        assert args.kernel_store == "chip", "the Phi_1 solve runs with --kernel-store chip (default) or wave"
        kernel_label, traffic_tag = ("fwd_vpair_kernel<3, true, true> (persistent O(v) point solve with the Phi_1 "
                                     "corrections, two points per wavefront)"), "fwd_vpair_kernel_nq32_ns3_phi1"
    elif args.kernel_store == "wave":
        launch.kernel_store = 5
        kernel_label, traffic_tag = ("fwd_v_kernel<3, true, false> (persistent O(v) point solve, one point per "
                                     "wavefront)"), "fwd_v_kernel_nq32_ns3"
    else:
        assert args.kernel_store == "chip", "the O(v) solve runs with --kernel-store chip (default) or wave"
        kernel_label, traffic_tag = ("fwd_vpair_kernel<3, true, false> (persistent O(v) point solve, two points per "
                                     "wavefront)"), "fwd_vpair_kernel_nq32_ns3"
    work = dict(D=D0.clone(), I=I0.clone(), ye=t["ye"].clone(), ef=ef0.clone(), v=t["v"].clone())
    outs = [S.alloc_outputs_v(model, P_POINTS, dev) for _ in range(STEPS_PER_GRAPH)]
    for o in outs:
        for k in work:
            o[k] = work[k]
    ws = S.PdarsWorkspace(model, P_POINTS, dev) if mode == "pdars" else S.Workspace(model, P_POINTS, dev)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(STEPS_PER_GRAPH)]
    step_fn = S.pdars_step_v if mode == "pdars" else S.solve_v

    def one_pass(record=False):
        work["D"].copy_(D0)
        work["I"].copy_(I0)
        work["ye"].copy_(t["ye"])
        work["ef"].copy_(ef0)
        work["v"].copy_(t["v"])
        for i in range(STEPS_PER_GRAPH):
            if record:
                ev[i][0].record()
            step_fn(model, params, W.DTAU_KM, work["D"], work["I"], t["rho11"], work["ye"], work["ef"],
                    work["v"], theta, out=outs[i], workspace=ws, launch=launch)
            if record:
                ev[i][1].record()

    one_pass()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        one_pass()
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    g0.record(stream)
    for _ in range(args.steps):
        g.replay()
    g1.record(stream)
    torch.cuda.synchronize()
    ms_per_step = 1e3 * (time.perf_counter() - t0) / args.steps
    graph_ms = g0.elapsed_time(g1) / args.steps
    # per launch: the replay's time on its stream less the pristine copy (as
    # for the static workload)
    cev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(5)]
    for a, b in cev:
        a.record(stream)
        work["D"].copy_(D0)
        work["I"].copy_(I0)
        work["ye"].copy_(t["ye"])
        work["ef"].copy_(ef0)
        work["v"].copy_(t["v"])
        b.record(stream)
    torch.cuda.synchronize()
    copy_ms = sorted(a.elapsed_time(b) for a, b in cev)[2]
    kern_ms = 0.0
    n_timed = max(2, min(args.steps, 5))
    for _ in range(n_timed):
        one_pass(record=True)
        torch.cuda.synchronize()
        kern_ms += sum(a.elapsed_time(b) for a, b in ev)
    n_in = np.stack([o["n_inner"].cpu().numpy() for o in outs]).astype(np.float64)
    n_out = np.stack([o["n_outer"].cpu().numpy() for o in outs]).astype(np.float64)
    status = np.stack([o["status"].cpu().numpy() for o in outs])
    solved = int(np.sum(n_out > 0))
    flops = float(np.sum((flops_per_point_v_phi1 if mode == "phi1" else flops_per_point_v)(n_in, n_out, 32)))
    eager_s = kern_ms * 1e-3 / (n_timed * STEPS_PER_GRAPH)
    kern_s = (graph_ms - copy_ms) * 1e-3 / STEPS_PER_GRAPH
    achieved = flops / STEPS_PER_GRAPH / kern_s / 1e12
    metric, unit, wl = {
        "solve": ("implicit O(v) point-solves/sec at 32 energy nodes, 3 species (FP64)", "point-solves/s",
                  "moving radial-profile (O(v) solve, fluid velocity up to 0.1 c), 2^16 points, 3 species, "
                  "32 energy nodes, full physics, 10 chained implicit steps per captured graph"),
        "phi1": ("implicit O(v) point-solves/sec with the Phi_1 corrections at 32 energy nodes, 3 species (FP64)",
                 "point-solves/s",
                 "moving radial-profile (O(v) solve with the linear-order Phi_1 NES and pair corrections, "
                 "Phi_1 = 0.3 / -0.25 Phi_0), 2^16 points, 3 species, 32 energy nodes, full physics, 10 chained "
                 "implicit steps per captured graph"),
        "pdars": ("PD-ARS coupling point-steps/sec at 32 energy nodes, 3 species (FP64)", "point-steps/s",
                  "moving radial-profile, one PD-ARS IMEX step of the coupling per step (O(v) solves with dt and "
                  "dt / 2, primitive recovery between them), 2^16 points, 3 species, 32 energy nodes, full physics, "
                  "10 chained steps per captured graph"),
    }[mode]
    line = {
        "metric": metric,
        "value": solved / (ms_per_step * 1e-3), "unit": unit, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {
            "workload": wl,
            "points": P_POINTS, "solved_point_steps_per_step": solved, "species": NS, "energy_nodes": 32,
            "implicit_steps_per_step": STEPS_PER_GRAPH, "dtau_km": W.DTAU_KM, "tol_inner": params.tol_inner,
            "tol_outer": params.tol_outer, "anderson_memory": params.m_inner,
            "launch": {"chunk": launch.chunk, "blocks_per_cu": launch.blocks_per_cu, "persistent": launch.persistent},
            "kernel_store": args.kernel_store,
            "iterations": iteration_summary(n_in, n_out),
            "status_counts": np.bincount(status.ravel(), minlength=5).tolist(),
        },
        "roofline": {
            "kernel": kernel_label + (" x 2 solves, with the recovery and stage kernels" if mode == "pdars" else ""),
            "flop_convention": {"solve": "O(v): closure and velocity work counted (flops_per_point_v)",
                                "phi1": "O(v) with the Phi_1 contractions and collision terms "
                                        "(flops_per_point_v_phi1)",
                                "pdars": "O(v) convention over both solves of the step (flops_per_point_v of the "
                                         "summed iteration counts); the recovery and stage work is not counted"}[mode],
            "bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS, "traffic": AT.stored_traffic(traffic_tag),
            "kernel_ms_per_launch": kern_s * 1e3,
            "kernel_ms_per_launch_from": ("graph replay time (HIP events, timed region) less the pristine copy, / 10"
                                          + ("; a launch is a whole PD-ARS step" if mode == "pdars" else "")),
            "graph_ms_per_step": graph_ms, "pristine_copy_ms": copy_ms, "eager_ms_per_launch": eager_s * 1e3,
            "flops_per_launch": flops / STEPS_PER_GRAPH,
            "algorithmic_hbm_gbs": bytes_per_point_v() * P_POINTS / kern_s / 1e9,
        },
    }
    from paper_2601_00976_amd import probe as PR
    fma_peak = PR.fma_tflops(dev)
    line["roofline"]["measured_fma_peak"] = fma_peak
    line["roofline"]["frac_of_measured_fma_peak"] = achieved / fma_peak
    if not args.no_cpu:
        threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
        line["cpu_baseline"] = cpu_baseline_v(args.cpu_steps_v, threads, mode)
    print(json.dumps(line), flush=True)


def run_c2p(args):
    """Primitive-moment recovery (Sec. 3.4) of every node of the moving
    profile: 2^16 points x 3 species x 32 nodes, the conserved moments (N, G)
    being the profile's drawn near-equilibrium moments at its fluid velocity
    (|v| up to 0.1), memory 3, tolerance 1e-8; 10 recoveries per captured
    graph."""
    import numpy as np
    import torch

    from paper_2601_00976_amd import autotune as AT
    from paper_2601_00976_amd import solver as S
    from paper_2601_00976_amd import workloads as W

    dev = torch.device("cuda:0")
    model = S.Model(S.Grid(16))
    t = S.to_device(W.radial_profile_v(P=P_POINTS, wid=V_WID), dev)
    Nc, G, _ = S.init_state_v(model, t)
    v = t["v"]
    cp = S.C2pParams()
    outs = [(torch.empty_like(Nc), torch.empty_like(G), torch.empty(Nc.shape, dtype=torch.int32, device=dev))
            for _ in range(STEPS_PER_GRAPH)]
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(STEPS_PER_GRAPH)]

    def one_pass(record=False):
        for i in range(STEPS_PER_GRAPH):
            if record:
                ev[i][0].record()
            S.primitive_recovery(model, Nc, G, v, cp, out=outs[i])
            if record:
                ev[i][1].record()

    one_pass()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        one_pass()
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    g0.record(stream)
    for _ in range(args.steps):
        g.replay()
    g1.record(stream)
    torch.cuda.synchronize()
    ms_per_step = 1e3 * (time.perf_counter() - t0) / args.steps
    graph_ms = g0.elapsed_time(g1) / args.steps
    kern_ms = 0.0
    n_timed = max(2, min(args.steps, 5))
    for _ in range(n_timed):
        one_pass(record=True)
        torch.cuda.synchronize()
        kern_ms += sum(a.elapsed_time(b) for a, b in ev)
    it = outs[0][2].cpu().numpy().astype(np.int64)
    nodes = int(it.size)
    assert np.all(it > 0), "a recovery hit its cap or went non-finite"
    kern_s = graph_ms * 1e-3 / STEPS_PER_GRAPH
    flops = float(np.sum(flops_per_node_c2p(it.astype(np.float64))))
    achieved = flops / kern_s / 1e12
    gbs = bytes_per_node_c2p() * nodes / kern_s / 1e9
    alu = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
           "frac": achieved / PEAK_FP64_TFLOPS}
    hbm = {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS}
    roof = alu if alu["frac"] >= hbm["frac"] else hbm
    other = hbm if roof is alu else alu
    line = {
        "metric": "primitive-moment recoveries/sec (nodes) at 32 energy nodes, 3 species (FP64)",
        "value": STEPS_PER_GRAPH * nodes / (ms_per_step * 1e-3), "unit": "node-recoveries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {
            "workload": "primitive-moment recovery of every node of the moving radial profile (2^16 points x 3 "
                        "species x 32 nodes, |v| up to 0.1), Anderson memory 3, tolerance 1e-8, 10 recoveries per "
                        "captured graph",
            "nodes": nodes, "recoveries_per_step": STEPS_PER_GRAPH, "anderson_memory": cp.mem, "tol": cp.tol,
            "iterations": {"min": int(it.min()), "median": float(np.median(it)), "max": int(it.max()),
                           "hist": np.bincount(it.ravel()).tolist()},
        },
        "roofline": dict(roof, kernel="c2p_kernel (one thread per node)",
                         flop_convention="flops_per_node_c2p: 158 per iteration + 30 per node",
                         traffic=AT.stored_traffic("c2p_kernel_nq32_ns3"), kernel_ms_per_launch=kern_s * 1e3,
                         kernel_ms_per_launch_from="graph replay time (HIP events, timed region) / 10",
                         eager_ms_per_launch=kern_ms / (n_timed * STEPS_PER_GRAPH), flops_per_launch=flops,
                         algorithmic_bytes_per_launch=bytes_per_node_c2p() * nodes,
                         other_bound={k: other[k] for k in ("bound", "achieved", "peak", "unit", "frac")}),
    }
    if not args.no_cpu:
        threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
        line["cpu_baseline"] = cpu_baseline_c2p(threads)
    print(json.dumps(line), flush=True)


def iteration_summary(n_in, n_out):
    """Iteration statistics of the solved point-steps, with histograms:
    inner_hist[k] / outer_hist[k] = point-steps with k inner / outer
    iterations."""
    import numpy as np

    solved = n_out > 0
    ni, no = n_in[solved].astype(np.int64), n_out[solved].astype(np.int64)
    return {"inner_min": int(ni.min()), "inner_median": float(np.median(ni)), "inner_max": int(ni.max()),
            "outer_median": float(np.median(no)), "outer_max": int(no.max()),
            "inner_hist": np.bincount(ni).tolist(), "outer_hist": np.bincount(no).tolist()}


def cpu_baseline(repeats: int, threads: int, all_points: bool = False):
    """The oracle (as it stands) on the same workload: the 10-step chain over
    all 2^16 profile points, repeated `repeats` times from the initial state,
    on `threads` host threads; then the chain over every 16th point on one
    thread.  Also returns the FLOPs of one chain priced from the oracle's own
    iteration counts (the convention of flops_per_point)."""
    import numpy as np

    import oracle as O
    from paper_2601_00976_amd import solver as S
    from paper_2601_00976_amd import workloads as W

    O.build(force=False)
    d = W.radial_profile(P=P_POINTS)
    m = O.Model(n_elem=16, overrides=dict(rho11_min=0.0) if all_points else {})
    theta = m.default_theta(S.DEFAULT_A_NES, S.DEFAULT_A_PAIR)

    def chain(dd, nthreads):
        D, I, e = m.init_state(dd.T, dd.rho11, dd.ye, dd.uD, dd.uI)
        ye = dd.ye.copy()
        solved, flops = 0, 0.0
        for _ in range(STEPS_PER_GRAPH):
            r = O.solve_batch(m, O.Params(), theta, W.DTAU_KM, D, I, dd.rho11, ye, e, nthreads=nthreads)
            D, I, ye, e = r["D"], r["I"], r["ye"], r["e"]
            solved += int(np.sum(r["n_outer"] > 0))
            flops += float(np.sum(flops_per_point(r["n_inner"].astype(np.float64),
                                                  r["n_outer"].astype(np.float64), 32)))
        return solved, flops

    solved, flops_chain = 0, 0.0
    t0 = time.perf_counter()
    for _ in range(repeats):
        s1, flops_chain = chain(d, threads)
        solved += s1
    dt = time.perf_counter() - t0
    sub = d.take(np.arange(0, P_POINTS, 16))
    t1 = time.perf_counter()
    solved1, _ = chain(sub, 1)
    dt1 = time.perf_counter() - t1
    # the oracle's own operation count (counting build) on every 64th profile
    # point of the first step, beside the convention's FLOPs for the same
    # point-solves
    O.build_tally(force=False)
    tp = d.take(np.arange(0, P_POINTS, 64))
    D0, I0, e0 = m.init_state(tp.T, tp.rho11, tp.ye, tp.uD, tp.uI)
    r, c = O.flop_tally(m, O.Params(), theta, W.DTAU_KM, D0, I0, tp.rho11, tp.ye, e0)
    conv = float(np.sum(flops_per_point(r["n_inner"].astype(np.float64), r["n_outer"].astype(np.float64), 32)))
    ora = c["add"] + c["mul"] + c["div"]
    tally = {"sample": f"every 64th profile point, step 1: {int(np.sum(r['n_outer'] > 0))} solves",
             "oracle_flops": ora, "convention_flops": conv, "oracle_over_convention": ora / conv,
             "oracle_sqrt": c["sqrt"], "oracle_transcendental_calls": c["trans"]}
    return dict(value=solved / dt, unit="point-solves/s", cores=threads, kind="oracle",
                sample=f"all {P_POINTS} profile points, {STEPS_PER_GRAPH} chained steps x {repeats}, "
                       f"{solved} solves in {dt:.1f} s",
                one_core={"value": solved1 / dt1, "unit": "point-solves/s", "cores": 1,
                          "sample": f"every 16th profile point, {STEPS_PER_GRAPH} chained steps, {solved1} solves "
                                    f"in {dt1:.1f} s"},
                flop_tally=tally, _flops_per_chain=flops_chain)


def adjoint_ratio(model, params, theta, D0, I0, t, e0, ws, launch, reps=5):
    """Adjoint versus forward cost on the first implicit step of the profile
    (loss weights gbar = (1, 1) per point), both eager on the same stream and
    timed with HIP events around each call."""
    import torch
    from paper_2601_00976_amd import solver as S
    from paper_2601_00976_amd import workloads as W

    P = D0.shape[0]
    out = S.alloc_outputs(model, P, D0.device)
    gbar = torch.ones(P, 2, dtype=torch.float64, device=D0.device)
    grad = torch.zeros(model.nq + 2, dtype=torch.float64, device=D0.device)

    def fwd():
        S.solve(model, params, W.DTAU_KM, D0, I0, t["rho11"], t["ye"], e0, theta, out=out, workspace=ws,
                launch=launch)

    def adj():
        S.adjoint(model, W.DTAU_KM, t["rho11"], theta, out, gbar, grad_theta=grad, workspace=ws)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        return sorted(a.elapsed_time(b) for a, b in ev)[reps // 2]

    t_f = timed(fwd)
    t_a = timed(adj)
    return {"workload": "radial profile step 1, 2^16 points, gbar = (1, 1)", "forward_ms": t_f, "adjoint_ms": t_a,
            "ratio": t_a / t_f}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-repeats", type=int, default=4, help="repeats of the 10-step chain in the oracle baseline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint-ratio leg (its step-1 forward launches would mix into a kernel profile)")
    ap.add_argument("--all-points", action="store_true",
                    help="solve every point of the profile (no low-density pass-through), down to T ~ 0.07 MeV")
    ap.add_argument("--fd-projection", action="store_true",
                    help="equilibrium by projection onto the energy elements with the bound-enforcing limiter "
                         "(the kernels' detailed balance from its odds) instead of pointwise Fermi-Dirac values")
    ap.add_argument("--chunk", type=int, default=None)
    ap.add_argument("--blocks-per-cu", type=int, default=None)
    ap.add_argument("--workload", choices=sorted(WORKLOADS) + ["profile-v", "profile-v-phi1", "pdars", "c2p"],
                    default="profile32",
                    help="profile32: the headline (2^16 points, 32 nodes); profile64: 2^18 points, 64 nodes; "
                         "profile-v: the O(v) solve on the moving profile (2^16 points, 32 nodes); profile-v-phi1: "
                         "the same with the linear-order Phi_1 corrections; pdars: PD-ARS IMEX steps of the "
                         "coupling on the moving profile; c2p: primitive-moment recovery of every node of the "
                         "moving profile")
    ap.add_argument("--cpu-steps-v", type=int, default=4, help="chained steps of the O(v) oracle baseline")
    ap.add_argument("--kernel-store", choices=("chip", "wave", "regen", "registers", "hbm"), default="chip",
                    help="chip: library default (32 nodes: two points per wavefront); wave (32 nodes): one point "
                         "per wavefront, pair factors in VGPRs; regen: kernel entries regenerated every inner "
                         "iteration; registers (32 nodes): rows held in VGPRs; hbm (64 nodes): kernels precomputed "
                         "in HBM")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the per-point solve needs no communication, and this "
              "build measures the single-GPU kernel (see the sharding notes in DESIGN.md).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2601_00976_amd import autotune as AT
    from paper_2601_00976_amd import solver as S
    from paper_2601_00976_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "profile-v":
        return run_velocity(args)
    if args.workload == "profile-v-phi1":
        return run_velocity(args, "phi1")
    if args.workload == "pdars":
        return run_velocity(args, "pdars")
    if args.workload == "c2p":
        return run_c2p(args)

    n_elem, P_POINTS, wid, traffic_tag, kernel_label = WORKLOADS[args.workload]
    nq = 2 * n_elem
    grid = S.Grid(n_elem)
    mkw = dict(rho11_min=0.0) if args.all_points else {}
    if args.fd_projection:
        assert nq == 32 and args.kernel_store == "chip", "--fd-projection runs in the 32-node two-point kernel"
        mkw["fd_projection"] = 1
        traffic_tag += "_proj"
        kernel_label = "fwd_pair_kernel<3,true,true> (two points per wavefront, projected equilibrium)"
    model = S.Model(grid, **mkw)
    params = S.Params()
    draws = W.radial_profile(P=P_POINTS, nq=nq, wid=wid)
    t = S.to_device(draws, dev)
    D0, I0, e0 = S.init_state(model, t["T"], t["rho11"], t["ye"], t["uD"], t["uI"])
    theta = model.default_theta()
    launch = AT.best_launch(model, P_POINTS)
    if args.chunk is not None:
        launch.chunk = args.chunk
    if args.blocks_per_cu is not None:
        launch.blocks_per_cu = args.blocks_per_cu
    hbm_store = args.kernel_store == "hbm"
    if args.kernel_store == "regen":
        assert nq == 32, "--kernel-store regen is the 64-node default; it is a mode of the 32-node solve"
        launch.kernel_store = 2
        traffic_tag = "fwd_kernel_nq32_ns3_regen"
        kernel_label = "fwd_kernel<3,32> (one point per wavefront, kernel entries regenerated)"
    if args.kernel_store == "registers":
        assert nq == 32, "--kernel-store registers needs --workload profile32"
        launch.kernel_store = 3
        traffic_tag = "fwd_kernel_nq32_ns3_registers"
        kernel_label = "fwd_kernel<3,32> (one point per wavefront, kernel rows held in VGPRs, DPP contraction)"
    if args.kernel_store == "wave":
        assert nq == 32, "--kernel-store wave needs --workload profile32"
        launch.kernel_store = 5
        traffic_tag = "fwd_kernel_nq32_ns3"
        kernel_label = "fwd_kernel<3,32> (one point per wavefront, pair factors in VGPRs)"
    if hbm_store:
        assert nq == 64, "--kernel-store hbm needs --workload profile64"
        launch.kernel_store = 1
        traffic_tag += "_hbm"
        kernel_label = "fwd64_kernel<3> (kernels precomputed per point in HBM)"

    # working state (solved in place step after step) and per-step counters
    work = dict(D=D0.clone(), I=I0.clone(), ye=t["ye"].clone(), e=e0.clone())
    outs = [S.alloc_outputs(model, P_POINTS, dev) for _ in range(STEPS_PER_GRAPH)]
    for o in outs:
        o["D"], o["I"], o["ye"], o["e"] = work["D"], work["I"], work["ye"], work["e"]
    ws = S.Workspace(model, P_POINTS, dev, kernel_store=hbm_store)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(STEPS_PER_GRAPH)]

    def one_pass(record=False):
        work["D"].copy_(D0)
        work["I"].copy_(I0)
        work["ye"].copy_(t["ye"])
        work["e"].copy_(e0)
        for i in range(STEPS_PER_GRAPH):
            if record:
                ev[i][0].record()
            S.solve(model, params, W.DTAU_KM, work["D"], work["I"], t["rho11"], work["ye"], work["e"], theta,
                    out=outs[i], workspace=ws, launch=launch)
            if record:
                ev[i][1].record()

    # eager warm-up (also caches the occupancy query outside capture)
    one_pass()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        one_pass()
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()

    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    g0.record(stream)
    for _ in range(args.steps):
        g.replay()
    g1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps
    graph_ms = g0.elapsed_time(g1) / args.steps

    # solve-kernel duration per launch: the graph replay's time on its stream
    # (HIP events over the timed region) less its pristine-state copy, per
    # launch; the remainder also holds the 10 counter-reset kernels (a few
    # microseconds each), so it slightly over-states the solve kernel
    def copies():
        work["D"].copy_(D0)
        work["I"].copy_(I0)
        work["ye"].copy_(t["ye"])
        work["e"].copy_(e0)

    cev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(5)]
    for a, b in cev:
        a.record(stream)
        copies()
        b.record(stream)
    torch.cuda.synchronize()
    copy_ms = sorted(a.elapsed_time(b) for a, b in cev)[2]
    kern_s_per_launch = (graph_ms - copy_ms) * 1e-3 / STEPS_PER_GRAPH
    # the same chain run eagerly with HIP events around every launch (reset
    # kernel, solve kernel and launch gaps), reported beside it
    kern_ms = 0.0
    n_timed = max(2, min(args.steps, 5))
    for _ in range(n_timed):
        one_pass(record=True)
        torch.cuda.synchronize()
        kern_ms += sum(a.elapsed_time(b) for a, b in ev)

    # accounting from the (deterministic) per-step iteration counts
    n_in = np.stack([o["n_inner"].cpu().numpy() for o in outs]).astype(np.float64)
    n_out = np.stack([o["n_outer"].cpu().numpy() for o in outs]).astype(np.float64)
    status = np.stack([o["status"].cpu().numpy() for o in outs])
    solved = int(np.sum(n_out > 0))
    flops = float(np.sum(flops_per_point(n_in, n_out, nq)))
    value = solved / (ms_per_step * 1e-3)
    eager_s_per_launch = kern_ms * 1e-3 / (n_timed * STEPS_PER_GRAPH)
    flops_per_launch = flops / STEPS_PER_GRAPH
    achieved = flops_per_launch / kern_s_per_launch / 1e12
    hbm_bytes_per_launch = bytes_per_point(nq) * P_POINTS
    traffic = AT.stored_traffic(traffic_tag)

    line = {
        "metric": f"implicit point-solves/sec at {nq} energy nodes, 3 species (FP64)",
        "value": value,
        "unit": "point-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"radial-profile, 2^{P_POINTS.bit_length() - 1} points, 3 species, {nq} energy nodes, "
                        "full physics, 10 chained implicit steps per captured graph",
            "points": P_POINTS, "solved_point_steps_per_step": solved, "species": NS, "energy_nodes": nq,
            "implicit_steps_per_step": STEPS_PER_GRAPH, "dtau_km": W.DTAU_KM, "tol": params.tol_inner,
            "kernel_store": args.kernel_store,
            "anderson_memory": params.m_inner, "launch": {"chunk": launch.chunk,
                                                          "blocks_per_cu": launch.blocks_per_cu,
                                                          "persistent": launch.persistent,
                                                          "autotune_key": AT.cache_key(model),
                                                          "from_cache": AT.cache_key(model) in AT.cache()},
            "iterations": iteration_summary(n_in, n_out),
            "status_counts": np.bincount(status.ravel(), minlength=5).tolist(),
            "all_points": bool(args.all_points),
            "fd_projection": bool(args.fd_projection),
        },
        "roofline": {
            "kernel": kernel_label,
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": traffic,
            "kernel_ms_per_launch": kern_s_per_launch * 1e3,
            "kernel_ms_per_launch_from": "graph replay time (HIP events, timed region) less the pristine copy, / 10",
            "graph_ms_per_step": graph_ms,
            "pristine_copy_ms": copy_ms,
            "eager_ms_per_launch": eager_s_per_launch * 1e3,
            "flops_per_launch": flops_per_launch,
            "algorithmic_hbm_gbs": hbm_bytes_per_launch / kern_s_per_launch / 1e9,
        },
    }
    # the denominator checked on this device: a pure FP64 FMA probe
    from paper_2601_00976_amd import probe as PR
    fma_peak = PR.fma_tflops(dev)
    line["roofline"]["measured_fma_peak"] = fma_peak
    line["roofline"]["frac_of_measured_fma_peak"] = achieved / fma_peak
    if nq == 32 and not args.no_adjoint and not args.all_points and not args.fd_projection:
        line["adjoint"] = adjoint_ratio(model, params, theta, D0, I0, t, e0, ws, launch)
    if not args.no_cpu and args.workload == "profile32" and not args.fd_projection:
        threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
        cb = cpu_baseline(args.cpu_repeats, threads, args.all_points)
        # the oracle's own iteration counts priced by the same convention:
        # FLOPs the GPU line claims per chain against those of the oracle
        cb["flops_per_chain"] = cb.pop("_flops_per_chain")
        cb["gpu_flops_per_chain"] = flops
        line["cpu_baseline"] = cb
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
