#!/usr/bin/env python3
"""Throughput benchmark of the WENO5 / HLLC / immersed-boundary / SSP-RK3 hot
path on one MI355X.

Default line: the largest single-GPU workload, the 2D Navier-Stokes Mach-3
shock on a circular cylinder (r = 0.1 at (0.3, 0.5)), ghost-cell immersed
boundary with a no-slip adiabatic wall, Re 1000, Pr 0.72, 1024 x 512 cells on
[0,2] x [0,1], FP64, automatic CFL-0.5 step.  An untimed approach carries the
shock onto the cylinder (t = 0.04; it meets the leading edge at t = 0.033),
then W untimed warm-up steps and K timed steps between two device
synchronisations, with the state resident in HBM.  One step = three fused
stage kernels (time step and ghost refill inside them).

The line carries the roofline of the dominant kernel (the stage kernel; its
launch durations are measured with HIP events on the stream it runs on), the
CPU oracle timed on a bounded sample of the same workload, and, as extra
keys, the 512^2 four-quadrant problem in FP64 and FP32, the same problem at
4096 x 2048 and 8192 x 4096 (HBM-resident sizes), the adjoint:forward cost
ratio and the learned correction's step cost and held-out error.
"""
import argparse
import gc
import json
import os
import sys
import time

METRIC = "cell-updates/s per RK3 step, % HBM peak; adjoint:forward cost ratio"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
# VALU issue ceiling: 256 CUs x 2.4 GHz x 64 lanes (four 16-lane SIMDs per CU,
# one wave-64 instruction per SIMD every four clocks), lane-instructions/s.
VALU_LANE_ISSUE_PER_S = 256 * 2.4e9 * 64
# Algorithmic arithmetic of one cell and one stage of the 2D Euler scheme
# (WENO5 on 4 variables at 2 faces, HLLC at 2 faces, primitive conversion,
# flux difference, stage combination), each +,-,*,/,sqrt,min,max counted once.
FLOPS_PER_CELL_STAGE = 1314
# Viscous stress and heat flux add about 45 operations per face (two faces
# per cell and stage) to the inviscid count.
FLOPS_PER_CELL_STAGE_VISCOUS = FLOPS_PER_CELL_STAGE + 90
# The characteristic-wise reconstruction adds per face: the Roe average and
# the eigenvector entries (~40), the conservative form of the six stencil
# cells (6 x 8), their projection (6 x 4 x 7), the back-projection of both
# states (2 x 28) and their primitives (2 x 8): ~330 per face, two faces per
# cell.
FLOPS_PER_CELL_STAGE_CHAR = FLOPS_PER_CELL_STAGE + 660
# HBM words per cell per step: stage 1 reads U and writes L(U) (8 words),
# stage 2 reads U and L(U) and writes U2, stage 3 reads U2 and U and writes U
# (12 words each).  With an immersed boundary each stage also reads the
# one-byte cell class.
WORDS_PER_CELL_STEP = 32
STAGE_SOURCES = ("stage.hip", "flux.hpp", "grid.hpp", "ibm_dev.hpp", "xcd.hpp", "mlp.hpp", "mlp_dev.hpp")
# Measured counters of the stage kernels (per dispatch, mean of the three
# stage modes): HBM bytes from FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (the
# copy-kernel calibration) and SQ_INSTS_VALU (wave instructions), for the
# stage-kernel sources whose SHA-256 is given; any other source or workload
# reports them as null.
MEASURED = {
    ("cylinder", 1024, 512, "f64"): {
        "sources_sha256": "ee20a6aafb7be9eba7ac01d63dc83a48fed7a726878a6761b89700f5eca0126f",
        "bytes_per_launch": 49866571, "valu_wave_instr_per_launch": 13305663,
        "profile": "profiles/stage_kernel_cylinder1024x512_ns_f64.md"},
    ("quadrant", 4096, 2048, "f64"): {
        "sources_sha256": "ee20a6aafb7be9eba7ac01d63dc83a48fed7a726878a6761b89700f5eca0126f",
        "bytes_per_launch": 803549911, "valu_wave_instr_per_launch": 186249713,
        "profile": "profiles/stage_kernel_quadrant4096x2048_f64.md"},
}


def stage_sources_sha256():
    """SHA-256 of the stage-kernel sources, or None where they are absent."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2601_04400_amd", "csrc")
    for f in STAGE_SOURCES:
        try:
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
        except OSError:
            return None
    return h.hexdigest()


def measured(key):
    m = MEASURED.get(key)
    if m is None or m["sources_sha256"] != stage_sources_sha256():
        return None
    return m


def roofline(n2, launch_s, flops_cell, bytes_cell, prec, key, kernel):
    """Roofline entry of the stage kernel: algorithmic bytes and flops per
    launch over the measured average launch duration, against the HBM and
    the vector-ALU peaks; the bound reported is the one with the larger
    fraction, the other is kept beside it with the VALU issue utilisation
    where counters for these sources were taken."""
    bytes_launch = bytes_cell * n2
    gbs = bytes_launch / launch_s / 1e9
    tflops = flops_cell * n2 / launch_s / 1e12
    fpeak = FP64_PEAK_TFLOPS if prec in ("f64", "mixed") else FP32_PEAK_TFLOPS
    m = measured(key)
    traffic = m["bytes_per_launch"] if m else None
    hbm = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic}
    alu = {"bound": "alu", "achieved": round(tflops, 2), "peak": fpeak, "unit": "TFLOP/s",
           "frac": round(tflops / fpeak, 4), "traffic": traffic}
    roof = dict(alu if alu["frac"] >= hbm["frac"] else hbm)
    roof["kernel"] = kernel
    roof["stage_us_per_launch"] = round(launch_s * 1e6, 3)
    roof["algorithmic_bytes_per_launch"] = bytes_launch
    roof["algorithmic_flops_per_launch"] = flops_cell * n2
    roof["other_bound"] = hbm if roof["bound"] == "alu" else alu
    if m:
        lane_instr = m["valu_wave_instr_per_launch"] * 64
        roof["valu_issue"] = {"lane_instr_per_cell_stage": round(lane_instr / n2, 1),
                              "frac_of_issue_ceiling": round(lane_instr / launch_s / VALU_LANE_ISSUE_PER_S, 4),
                              "profile": m["profile"]}
    return roof


def cpu_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(nx, ny, budget_s):
    """The oracle (serial FP64 C++), timed on a bounded number of RK3 steps of
    the same problem from the same initial state."""
    import oracle
    oracle.threads(1)  # the serial oracle
    from paper_2601_04400_amd import inputs
    c = oracle.config(nx=nx, ny=ny)
    U = oracle.prim_to_cons(c, inputs.riemann2d_prim(nx, ny))
    t0 = time.perf_counter()
    U1, _, s1, _ = oracle.run(c, U, 1e30, max_steps=1)
    one = time.perf_counter() - t0
    steps = max(1, int(budget_s / max(one, 1e-6)))
    t0 = time.perf_counter()
    _, _, s, _ = oracle.run(c, U, 1e30, max_steps=steps)
    el = time.perf_counter() - t0
    model, ncpu = cpu_info()
    return {"value": nx * ny * s / el, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{s} automatic RK3 steps of the {nx}x{ny} four-quadrant problem from t=0 "
                      f"({el:.1f} s, serial FP64 oracle, 1 thread of {ncpu} on '{model}')"}


def adjoint_ratio(n=256, steps=200, every=20):
    """Adjoint:forward cost on the inviscid shock-cylinder sensitivity problem
    (256^2, 200 fixed steps, checkpoints every 20): wall time of the backward
    pass (segment replays included) over the forward pass, the median of
    five measured repetitions after a warm-up one; with the replays on a
    replica grid overlapping the reverse pass (reported) and in one stream
    (serial_replay)."""
    import torch
    from paper_2601_04400_amd import Grid, inputs, normal_shock_state
    from paper_2601_04400_amd.adjoint import rollout
    dom = (0.0, 1.0, 0.0, 1.0)
    phi = inputs.circle_phi(n, n, dom, (0.3, 0.5), 0.1)
    post, _, _ = normal_shock_state(3.0)
    inflow = (post[0], post[1], 0.0, post[2])
    g = Grid(n, n, domain=dom, bc=(2, 0, 1, 1), inflow=inflow, ibm=True, adjoint=True)
    g.set_levelset(torch.from_numpy(phi), wall=0)
    U0 = g.prim_to_cons(torch.from_numpy(inputs.shock_prim(n, n, dom, 0.1, inflow, (1.4, 0, 0, 1))))
    d = torch.zeros(1, dtype=torch.float64, device="cuda")
    g.set_time(0.0, 1.0)
    g.step(U0.clone(), dt_out=d)
    dt = 0.6 * float(d.cpu()[0])
    params = torch.tensor([[1.4, *inflow]], dtype=torch.float64, device="cuda", requires_grad=True)

    def measure(overlap):
        # the timed repetitions run with Python's garbage collector paused
        gc.collect()
        gc.disable()
        try:
            return _measure(overlap)
        finally:
            gc.enable()

    def _measure(overlap):
        runs = []
        for rep in range(6):  # the first is a warm-up; the median and the maximum of the other five are reported
            # both gradients start empty in every repetition: accumulating into
            # an existing params.grad would run torch's own add kernel, whose
            # first (lazy) load stalled one repetition's backward call by
            # ~65 ms after the library's work had been issued
            U0.grad = None
            params.grad = None
            U0.requires_grad_(True)
            trace = [] if overlap else None
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            U = rollout(g, U0, params, steps, dt, every, overlap=overlap, trace=trace)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            b0, b1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            b0.record()
            U.backward(torch.ones_like(U))
            b1.record()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            if rep > 0:
                tl = timeline(b0, trace) or {}
                tl["backward_gpu_ms"] = round(b0.elapsed_time(b1), 3)
                runs.append(((t2 - t1) / (t1 - t0), t1 - t0, t2 - t1, tl))
        runs.sort(key=lambda r: r[0])
        return runs

    def timeline(b0, trace):
        """Milliseconds from the backward pass's start to each traced event,
        and the summed durations of the replays, the reverse segments and the
        main stream's waits for a replay."""
        if not trace:
            return {}
        at = {lab: b0.elapsed_time(e) for lab, e in trace}
        segs = sorted({int(lab.split()[1]) for lab in at})
        rep_ms = sum(at[f"replay {c} end"] - at[f"replay {c} start"] for c in segs)
        rev_ms = sum(at[f"reverse {c} end"] - at[f"reverse {c} start"] for c in segs)
        wait_ms = sum(max(0.0, at[f"reverse {c} start"] - max(at[f"reverse {c} issued"],
                                                             at.get(f"reverse {c + 1} end", 0.0))) for c in segs)
        return {"replays_ms": round(rep_ms, 3), "reverse_ms": round(rev_ms, 3), "main_waits_ms": round(wait_ms, 3),
                "events_ms": {lab: round(v, 3) for lab, v in at.items()}}

    runs = measure(True)
    serial = measure(False)
    r, f, b, _ = runs[len(runs) // 2]
    rs, fs, bs, _ = serial[len(serial) // 2]
    worst = runs[-1]
    res = {"forward_ms": round(f * 1e3, 3), "backward_ms": round(b * 1e3, 3), "ratio": round(r, 3),
           "ratio_max": round(worst[0], 3), "repetitions": len(runs),
           "measured_fwd_bwd_ms": [[round(x[1] * 1e3, 3), round(x[2] * 1e3, 3)] for x in runs],
           "timeline_median": {k: v for k, v in runs[len(runs) // 2][3].items() if k != "events_ms"},
           "timeline_max": runs[-1][3],
           "serial_replay": {"forward_ms": round(fs * 1e3, 3), "backward_ms": round(bs * 1e3, 3),
                             "ratio": round(rs, 3), "ratio_max": round(serial[-1][0], 3)}}
    res["workload"] = (f"inviscid Mach-3 shock on a cylinder, {n}x{n}, {steps} fixed RK3 steps, "
                       f"checkpoint every {every}, slip immersed boundary; backward includes segment replays "
                       f"(on a replica grid and second stream, overlapping the reverse pass; serial_replay: "
                       f"the same backward with replays and reverse steps in one stream)")
    return res


def copy_ceiling(mb=512, reps=10):
    """Measured device-copy bandwidth (read + write bytes per second) of a
    plain torch copy of `mb` MiB, HIP-event timed: the practical HBM ceiling."""
    import torch
    a = torch.ones(mb * 2 ** 20 // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * a.numel() * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    return round(gbs, 1)


CYL_NX, CYL_NY = 1024, 512
CYL_T_AT_BODY = 0.04  # the shock (speed 3 from x = 0.1) passes the cylinder's leading edge x = 0.2 at t = 0.033


def cylinder_problem(nx=CYL_NX, ny=CYL_NY, xs=0.1):
    """Set-up of the viscous shock-cylinder case: primitive state, level set,
    boundary rules, inflow state and viscosity (Re 1000 on the diameter)."""
    from paper_2601_04400_amd import inputs, normal_shock_state
    dom = (0.0, 2.0, 0.0, 1.0)
    post, _, _ = normal_shock_state(3.0)
    inflow = (post[0], post[1], 0.0, post[2])
    sc = inputs.shock_cylinder(nx, ny, inflow, domain=dom, centre=(0.3, 0.5), radius=0.1, xs=xs)
    return sc, inflow, inputs.cylinder_viscosity(3.0)


def cylinder_workload(args):
    """The headline workload (module docstring): approach to the body, W
    warm-up steps, K timed steps (wall clock and HIP events on the stream
    the stage kernels run on), then the same K steps with an event pair
    around every kernel for the per-stage breakdown."""
    import torch
    from paper_2601_04400_amd import Grid
    nx, ny, K, W = CYL_NX, CYL_NY, args.steps, args.warmup
    sc, inflow, mu = cylinder_problem()
    g = Grid(nx, ny, domain=sc["domain"], bc=sc["bc"], inflow=inflow, ibm=True, viscous=True, mu=mu, prandtl=0.72)
    nghost = g.set_levelset(torch.from_numpy(sc["phi"]), wall=1)
    U = g.prim_to_cons(torch.from_numpy(sc["W"]))
    t_body, approach = g.advance(U, CYL_T_AT_BODY, chunk=8)  # at most 7 no-op steps after the body is reached
    g.set_time(t_body, 1e30)  # no end time inside the measured run
    for _ in range(W):
        g.step(U)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(K):
        g.step(U)
    ev1.record()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    t_end_timed, _, steps_end = g.get_time()
    g.profile(True)
    for _ in range(K):
        g.step(U)
    prof = g.profile_read()
    g.profile(False)
    flags, fb = g.poll_faults()
    n2 = nx * ny
    # the timed region holds exactly 3 K stage launches and nothing else
    launch_s = gpu_ms * 1e-3 / (3 * K)
    roof = roofline(n2, launch_s, FLOPS_PER_CELL_STAGE_VISCOUS, WORDS_PER_CELL_STEP * 8 / 3 + 1, "f64",
                    ("cylinder", nx, ny, "f64"), "stage_kernel, viscous immersed-boundary variant (3 launches per step)")
    roof["launches_timed"] = 3 * K
    return {
        "metric": METRIC, "value": n2 * K / el, "unit": "cell-updates/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": el * 1e3 / K, "gpu_ms_per_step": gpu_ms / K, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "2D Navier-Stokes Mach-3 shock on a cylinder r=0.1 at (0.3,0.5), ghost-cell IBM, "
                               "no-slip adiabatic wall, Re 1000, Pr 0.72, 1024x512 on [0,2]x[0,1], WENO5-JS+HLLC, "
                               "SSP-RK3, CFL 0.5, FP64; timed after the shock has reached the cylinder",
                   "nx": nx, "ny": ny, "ghost_cells": nghost, "approach_steps": approach,
                   "t_timed": [round(t_body, 5), round(t_end_timed, 5)]},
        "hbm_frac_of_peak": round(WORDS_PER_CELL_STEP * 8 * n2 * K / el / 1e9 / HBM_PEAK_GBS, 4),
        "roofline": roof,
        "kernel_ms_event_bracketed": {k: round(v[0] / max(v[1], 1), 5) for k, v in prof.items() if v[1]},
        "faults": {"flags": flags, "fallback_faces": fb}, "device_steps": steps_end,
    }


def cylinder_cpu_baseline(budget_s):
    """The oracle (serial FP64 C++) on the same grid, level set, wall and
    viscosity, from a state with the shock already at the cylinder (the
    planar shock placed at x = 0.25, inside the cylinder's leading part), for
    about budget_s seconds of automatic steps."""
    import oracle
    oracle.threads(1)  # the serial oracle
    nx, ny = CYL_NX, CYL_NY
    sc, inflow, mu = cylinder_problem(xs=0.25)
    c = oracle.config(nx=nx, ny=ny, x0=0.0, x1=2.0, y0=0.0, y1=1.0, viscous=1, mu=mu, prandtl=0.72, bc=sc["bc"],
                      inflow=inflow)
    U = oracle.prim_to_cons(c, sc["W"])
    t0 = time.perf_counter()
    oracle.run(c, U, 1e30, max_steps=1, phi=sc["phi"], wall=1)
    one = time.perf_counter() - t0
    steps = max(1, int(budget_s / max(one, 1e-6)))
    t0 = time.perf_counter()
    _, _, s, _ = oracle.run(c, U, 1e30, max_steps=steps, phi=sc["phi"], wall=1)
    el = time.perf_counter() - t0
    model, ncpu = cpu_info()
    return {"value": nx * ny * s / el, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{s} automatic RK3 steps of the 1024x512 viscous shock-cylinder case from a state with the "
                      f"shock at the cylinder ({el:.1f} s, serial FP64 oracle, 1 thread of {ncpu} on '{model}')"}


def quadrant_run(nx, ny, prec="f64", K=300, W=30, char=False, graph=False):
    """The four-quadrant Riemann problem (seeded +-5 % quadrant states,
    transmissive): W warm-up steps, K timed automatic steps (three fused stage
    launches each, nothing else), the stage kernel's roofline."""
    import torch
    from paper_2601_04400_amd import Grid, inputs
    n2 = nx * ny
    g = Grid(nx, ny, prec=prec, weno_char=char)
    U = g.prim_to_cons(torch.from_numpy(inputs.riemann2d_prim(nx, ny)))
    g.set_time(0.0, 1e30)  # no end time inside the run: every step is a full step
    for _ in range(W):
        g.step(U)
    torch.cuda.synchronize()
    cg = None
    if graph:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            g.step(U)
        torch.cuda.current_stream().wait_stream(s)
        cg = torch.cuda.CUDAGraph()
        with torch.cuda.graph(cg):
            for _ in range(K):
                g.step(U)
        torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    if cg is not None:
        cg.replay()
    else:
        for _ in range(K):
            g.step(U)
    ev1.record()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    flags, fb = g.poll_faults()
    esize = 8 if prec == "f64" else 4
    launch_s = gpu_ms * 1e-3 / (3 * K)
    flops_cell = FLOPS_PER_CELL_STAGE_CHAR if char else FLOPS_PER_CELL_STAGE
    roof = roofline(n2, launch_s, flops_cell, WORDS_PER_CELL_STEP * esize / 3, prec,
                    ("quadrant", nx, ny, prec) if not char else None, "stage_kernel (3 launches per step)")
    roof["launches_timed"] = 3 * K
    del g, U
    return {"value": n2 * K / el, "unit": "cell-updates/s", "ms_per_step": el * 1e3 / K, "gpu_ms_per_step": gpu_ms / K,
            "steps": K, "warmup": W, "dtype": prec,
            "hbm_frac_of_peak": round(WORDS_PER_CELL_STEP * esize * n2 * K / el / 1e9 / HBM_PEAK_GBS, 4),
            "roofline": roof, "faults": {"flags": flags, "fallback_faces": fb},
            "workload": f"2D Euler four-quadrant Riemann problem {nx}x{ny} on [0,1]^2, gamma 1.4, seeded +-5% "
                        "quadrant states, transmissive, " + ("characteristic-wise " if char else "")
                        + f"WENO5-JS+HLLC, SSP-RK3, CFL 0.5, {prec.upper()}"}


def learned_costs(iters=400):
    """The learned correction on its workload: 64 seeded four-quadrant
    problems at 128^2 against 512^2 restricted 4x4, the per-face network
    trained from zero output for `iters` Adam iterations (unrolled m = 16),
    then the held-out problems (seeds 1000-1015): mean squared error after
    24 coarse steps and the cost per coarse step, with and without the
    correction, and of the finer solvers."""
    import torch
    from paper_2601_04400_amd import learn as L
    t0 = time.perf_counter()
    data = L.Dataset(list(range(64)), nc=128, factor=4, nsnap=24)
    net = L.FluxNet(L.init_theta(0, zero_output=True))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L.train(net, data, iters=iters, m=16)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    ev = L.evaluate(net, list(range(1000, 1016)), nc=128, factor=4, nsteps=24)
    keep = {k: {kk: (round(vv, 9) if isinstance(vv, float) else vv) for kk, vv in v.items()}
            for k, v in ev.items() if k not in ("learned", "plain")}
    return {"workload": "per-face MLP correction, 64 training problems 128^2 vs 512^2 restricted 4x4, m = 16, "
                        f"{iters} Adam iterations (1e-3, then 1e-4 for the last eighth); 16 held-out problems, "
                        "24 coarse steps",
            "train_ms_per_iter": round(train_s * 1e3 / iters, 3), "total_s": round(time.perf_counter() - t0, 2),
            "heldout": keep}


def sod_cpu_baseline():
    """The oracle on the whole Sod run (200 cells to t = 0.2)."""
    import oracle
    oracle.threads(1)  # the serial oracle
    from paper_2601_04400_amd import inputs
    c = oracle.config(ndim=1, nx=200)
    U = oracle.prim_to_cons(c, inputs.sod_prim(200))
    t0 = time.perf_counter()
    _, _, steps, _ = oracle.run(c, U, 0.2)
    el = time.perf_counter() - t0
    model, ncpu = cpu_info()
    return {"value": 200 * steps / el, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "time_to_solution_ms": round(el * 1e3, 3),
            "sample": f"the whole run ({steps} steps, serial FP64 oracle, 1 thread of {ncpu} on '{model}')"}


def paper_cylinder_workload(args):
    """The paper's Mach-5 shock-cylinder run at its largest size: 4096 x 2048
    on [-0.5, 4] x [0, 2] (8.4e6 cells), slip immersed boundary, inflow /
    outflow / reflective walls, FP64, automatic CFL-0.5 step, from t = 0 to
    t = 1.2: time to solution with the state resident on the GPU."""
    import torch
    from paper_2601_04400_amd import Grid, inputs
    nx, ny, t_end = 4096, 2048, 1.2
    sc = inputs.paper_shock_cylinder(nx, ny)
    g = Grid(nx, ny, domain=sc["domain"], bc=sc["bc"], inflow=sc["inflow"], ibm=True)
    nghost = g.set_levelset(torch.from_numpy(sc["phi"]), wall=0)
    U = g.prim_to_cons(torch.from_numpy(sc["W"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t, steps = g.advance(U, t_end, chunk=256)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    flags, fb = g.poll_faults()
    n2 = nx * ny
    return {
        "metric": METRIC, "value": n2 * steps / el, "unit": "cell-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": 0, "ms_per_step": el * 1e3 / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "2D Euler Mach-5 shock on a cylinder r=0.25 at (0.6,1), [-0.5,4]x[0,2], 4096x2048, "
                               "slip ghost-cell IBM, inflow/outflow/reflective, CFL 0.5, t 0 to 1.2, FP64",
                   "nx": nx, "ny": ny, "ghost_cells": nghost},
        "time_to_solution_s": round(el, 3), "t_reached": t,
        "faults": {"flags": flags, "fallback_faces": fb},
        "context": "the paper times this run at 1350 s on an H100 NVL and 10354 s on an RTX A6000 "
                   "(precision not stated); other hardware, not a target",
    }


def sod_workload(args):
    """1D Euler Sod shock tube, 200 cells on [0,1], transmissive, CFL 0.5,
    to t = 0.2, FP64: time to solution from a resident state (latency-bound:
    a few microseconds per launch), repeated reps times."""
    import torch
    from paper_2601_04400_amd import Grid, inputs
    n, reps = 200, 20
    g = Grid(n, ndim=1)
    W = torch.from_numpy(inputs.sod_prim(n))
    U0 = g.prim_to_cons(W)
    U = U0.clone()
    t, steps = g.advance(U, 0.2)  # warm-up and step count
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(reps):
        U.copy_(U0)
        g.set_time(0.0, 0.2)
        for _ in range(steps):
            g.step(U)
    ev1.record()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    gpu_s = ev0.elapsed_time(ev1) * 1e-3 / reps
    tt, done, st2 = g.get_time()
    return {
        "metric": METRIC, "value": n * steps / el, "unit": "cell-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": 1, "ms_per_step": el * 1e3 / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "1D Euler Sod shock tube, 200 cells on [0,1], gamma 1.4, transmissive, WENO5-JS+HLLC, "
                               "SSP-RK3, CFL 0.5, t_end 0.2, FP64", "nx": n},
        "time_to_solution_ms": round(el * 1e3, 3), "gpu_time_to_solution_ms": round(gpu_s * 1e3, 3),
        "t_reached": tt, "done": done, "note": "launch-latency bound; not a bandwidth or ALU measurement",
        "cpu_baseline": None if args.no_cpu_baseline else sod_cpu_baseline(),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--workload", default="cylinder",
                    choices=["cylinder", "quadrant", "sod", "paper-cylinder", "adjoint"],
                    help="cylinder: the viscous shock-cylinder case at 1024x512 (default, with the extra keys); "
                         "quadrant: the four-quadrant Riemann problem (--nx, --ny, --prec, --weno, --graph); "
                         "sod: the 200-cell shock tube; paper-cylinder: the section 3 run at 4096x2048; "
                         "adjoint: the adjoint:forward measurement alone (each prints its own line)")
    ap.add_argument("--nx", type=int, default=512, help="quadrant: cells along x")
    ap.add_argument("--ny", type=int, default=512, help="quadrant: cells along y")
    ap.add_argument("--prec", default="f64", choices=["f64", "f32", "mixed"], help="quadrant: precision")
    ap.add_argument("--weno", default="prim", choices=["prim", "char"],
                    help="quadrant: WENO5 on primitive (default) or characteristic variables (FP64)")
    ap.add_argument("--graph", action="store_true", help="quadrant: replay the timed steps from a HIP graph")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MB",
                    help="instead: time a plain device copy of MB megabytes (counter calibration)")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle time")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="cylinder: only the headline (no 512^2, at-scale, adjoint or learned-correction keys)")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint:forward cost measurement")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-correction measurement")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(the path would shard by spatial slabs with a 3-cell halo exchange per stage)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_probe:
        nbytes = args.copy_probe * 2 ** 20
        a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        print(json.dumps({"copy_probe_bytes_read": nbytes, "copy_probe_bytes_written": nbytes,
                          "copies": args.steps, "GB_per_s": 2 * nbytes * args.steps / el / 1e9}), flush=True)
        return

    if args.workload == "sod":
        print(json.dumps(sod_workload(args)), flush=True)
        return
    if args.workload == "paper-cylinder":
        print(json.dumps(paper_cylinder_workload(args)), flush=True)
        return
    if args.workload == "adjoint":
        # the adjoint:forward measurement of the default line on its own
        res = adjoint_ratio()
        print(json.dumps({"metric": "adjoint:forward cost ratio", "value": res["ratio"], "unit": "ratio",
                          "n_gpus": 1, "higher_is_better": False, "dtype": "f64", "data": "synthetic",
                          "config": {"workload": res["workload"]}, "adjoint": res}), flush=True)
        return
    if args.workload == "quadrant":
        q = quadrant_run(args.nx, args.ny, args.prec, args.steps, args.warmup, args.weno == "char", args.graph)
        out = {"metric": METRIC, "value": q.pop("value"), "unit": q.pop("unit"), "n_gpus": 1, "steps": q.pop("steps"),
               "warmup": q.pop("warmup"), "ms_per_step": q.pop("ms_per_step"), "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": q.pop("dtype"), "data": "synthetic",
               "config": {"workload": q.pop("workload"), "nx": args.nx, "ny": args.ny, "prec": args.prec,
                          "graph": bool(args.graph), "weno": args.weno}}
        out.update(q)
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(args.nx, args.ny, args.cpu_budget)
        print(json.dumps(out), flush=True)
        return

    out = cylinder_workload(args)
    print("bench: headline measured", file=sys.stderr, flush=True)
    if not args.no_extras:
        out["hbm_copy_ceiling_GBs"] = copy_ceiling()
        out["quadrant_512"] = {p: quadrant_run(512, 512, p) for p in ("f64", "f32")}
        print("bench: 512^2 measured", file=sys.stderr, flush=True)
        out["at_scale"] = {f"{nx}x{ny}": quadrant_run(nx, ny, "f64", K=60, W=5)
                           for nx, ny in ((4096, 2048), (8192, 4096))}
        print("bench: at-scale grids measured", file=sys.stderr, flush=True)
        if not args.no_adjoint:
            out["adjoint"] = adjoint_ratio()
            print("bench: adjoint measured", file=sys.stderr, flush=True)
        if not args.no_learned:
            out["learned_correction"] = learned_costs()
            print("bench: learned correction measured", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cylinder_cpu_baseline(args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
