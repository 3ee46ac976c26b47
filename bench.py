#!/usr/bin/env python3
"""Throughput benchmark of the WENO5 / HLLC / SSP-RK3 hot path on one MI355X.

Workload (default): 2D Euler four-quadrant Riemann problem, 512 x 512 cells on
[0,1]^2, gamma 1.4, seeded +-5 % piecewise-constant quadrant states,
transmissive boundaries, WENO5-JS + HLLC, SSP-RK3 with the automatic CFL-0.5
step, FP64.  One step = CFL reduction + three fused stage kernels.  The state
starts resident in HBM; W untimed warm-up steps, then K timed steps between
two device synchronisations.

Prints ONE JSON line with the metric, the roofline of the dominant kernel
(the fused stage kernel; its launch durations are measured with HIP events
on the stream it runs on, in a second pass of the same K steps) and the CPU
oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

METRIC = "cell-updates/s per RK3 step, % HBM peak; adjoint:forward cost ratio"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
# Algorithmic arithmetic of one cell and one stage of the 2D Euler scheme
# (WENO5 on 4 variables at 2 faces, HLLC at 2 faces, primitive conversion,
# flux difference, stage combination), each +,-,*,/,sqrt,min,max counted once.
FLOPS_PER_CELL_STAGE = 1314
# HBM words per cell per step: stage 1 reads U and writes U1 (8 words),
# stages 2 and 3 read U_s and U^n and write U_{s+1} (12 words each).
WORDS_PER_CELL_STEP = 32
# Measured HBM traffic of the fused stage kernels (FETCH_SIZE and WRITE_SIZE
# per dispatch, mean of the three stage modes, bytes), scaled by the copy-
# kernel calibration (fetch x 2.0, write x 1.0), for the stage-kernel sources
# whose SHA-256 is given; reported as null for any other source or workload.
MEASURED_TRAFFIC = {
    "sources_sha256": "e8073d88652adc2b9d259b7b140f3afb44c523a35e6609b3d8cdd13332d5d908",
    "workload": (512, 512, "f64"),
    "bytes_per_launch": 23512390,
    "profile": "profiles/stage_kernel_quadrant512_f64.md",
}
STAGE_SOURCES = ("stage.hip", "flux.hpp", "xcd.hpp")


def stage_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2601_04400_amd", "csrc")
    for f in STAGE_SOURCES:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


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
        runs = []
        for rep in range(6):  # the first is a warm-up; the median of the other five is reported
            U0.grad = None
            U0.requires_grad_(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            U = rollout(g, U0, params, steps, dt, every, overlap=overlap)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            U.backward(torch.ones_like(U))
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            if rep > 0:
                runs.append(((t2 - t1) / (t1 - t0), t1 - t0, t2 - t1))
        runs.sort()
        return runs

    runs = measure(True)
    serial = measure(False)
    r, f, b = runs[len(runs) // 2]
    rs, fs, bs = serial[len(serial) // 2]
    res = {"forward_ms": round(f * 1e3, 3), "backward_ms": round(b * 1e3, 3), "ratio": round(r, 3),
           "measured_fwd_bwd_ms": [[round(x[1] * 1e3, 3), round(x[2] * 1e3, 3)] for x in runs],
           "serial_replay": {"forward_ms": round(fs * 1e3, 3), "backward_ms": round(bs * 1e3, 3),
                             "ratio": round(rs, 3)}}
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


# Viscous stress and heat flux add about 45 operations per face (two faces
# per cell and stage) to the inviscid count.
FLOPS_PER_CELL_STAGE_VISCOUS = FLOPS_PER_CELL_STAGE + 90
# The characteristic-wise reconstruction adds per face: the Roe average and
# the eigenvector entries (~40), the conservative form of the six stencil
# cells (6 x 8), their projection (6 x 4 x 7), the back-projection of both
# states (2 x 28) and their primitives (2 x 8): ~330 per face, two faces per
# cell.
FLOPS_PER_CELL_STAGE_CHAR = FLOPS_PER_CELL_STAGE + 660


def cylinder_workload(args):
    """Navier-Stokes Mach-3 planar shock on a circular cylinder (r = 0.1 at
    (0.3, 0.5)) by the ghost-cell immersed boundary, no-slip adiabatic wall,
    Re = 1000 on the diameter, Pr = 0.72, 1024 x 512 on [0,2] x [0,1], FP64,
    automatic CFL-0.5 step; W untimed steps take the shock onto the cylinder,
    then K timed steps.  One step = CFL reduction + 3 x (refill + stage)."""
    import torch
    from paper_2601_04400_amd import Grid, inputs, normal_shock_state
    nx, ny, K, W = 1024, 512, args.steps, args.warmup
    dom = (0.0, 2.0, 0.0, 1.0)
    post, _, _ = normal_shock_state(3.0)
    inflow = (post[0], post[1], 0.0, post[2])
    sc = inputs.shock_cylinder(nx, ny, inflow, domain=dom, centre=(0.3, 0.5), radius=0.1, xs=0.1)
    g = Grid(nx, ny, domain=dom, bc=sc["bc"], inflow=inflow, ibm=True, viscous=True,
             mu=inputs.cylinder_viscosity(3.0), prandtl=0.72)
    nghost = g.set_levelset(torch.from_numpy(sc["phi"]), wall=1)
    U = g.prim_to_cons(torch.from_numpy(sc["W"]))
    g.set_time(0.0, 1e30)
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
    g.profile(True)
    for _ in range(K):
        g.step(U)
    prof = g.profile_read()
    g.profile(False)
    flags, fb = g.poll_faults()
    t, _, steps = g.get_time()
    n2 = nx * ny
    stage_s = sum(prof[k][0] for k in ("stage1", "stage2", "stage3")) * 1e-3 / (3 * K)
    tflops = FLOPS_PER_CELL_STAGE_VISCOUS * n2 / stage_s / 1e12
    return {
        "metric": METRIC, "value": n2 * K / el, "unit": "cell-updates/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": el * 1e3 / K, "gpu_ms_per_step": gpu_ms / K, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "2D Navier-Stokes Mach-3 shock on a cylinder r=0.1 at (0.3,0.5), ghost-cell IBM, "
                               "no-slip adiabatic, Re 1000, Pr 0.72, 1024x512 on [0,2]x[0,1], CFL 0.5, timed "
                               f"after {W} steps (t = {t:.4f} at the end of the run)",
                   "nx": nx, "ny": ny, "ghost_cells": nghost},
        "stage_kernel": {"us_per_launch_event_bracketed": round(stage_s * 1e6, 3),
                         "alu_TFLOPs": round(tflops, 2), "alu_frac": round(tflops / FP64_PEAK_TFLOPS, 4)},
        "kernel_ms_event_bracketed": {k: round(v[0] / max(v[1], 1), 5) for k, v in prof.items() if v[1]},
        "faults": {"flags": flags, "fallback_faces": fb}, "device_steps": steps,
        "cpu_baseline": None if args.no_cpu_baseline else cylinder_cpu_baseline(),
    }


def sod_cpu_baseline():
    """The oracle on the whole Sod run (200 cells to t = 0.2)."""
    import oracle
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


def cylinder_cpu_baseline(steps=6):
    """The oracle on a few steps of the viscous shock-cylinder case from its
    initial state (the same grid, level set and wall)."""
    import oracle
    from paper_2601_04400_amd import inputs, normal_shock_state
    nx, ny = 1024, 512
    dom = (0.0, 2.0, 0.0, 1.0)
    post, _, _ = normal_shock_state(3.0)
    inflow = (post[0], post[1], 0.0, post[2])
    sc = inputs.shock_cylinder(nx, ny, inflow, domain=dom, centre=(0.3, 0.5), radius=0.1, xs=0.1)
    c = oracle.config(nx=nx, ny=ny, x0=0.0, x1=2.0, y0=0.0, y1=1.0, viscous=1, mu=inputs.cylinder_viscosity(3.0),
                      prandtl=0.72, bc=sc["bc"], inflow=inflow)
    U = oracle.prim_to_cons(c, sc["W"])
    t0 = time.perf_counter()
    _, _, s, _ = oracle.run(c, U, 1e30, max_steps=steps, phi=sc["phi"], wall=1)
    el = time.perf_counter() - t0
    model, ncpu = cpu_info()
    return {"value": nx * ny * s / el, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{s} automatic RK3 steps from the initial state ({el:.1f} s, serial FP64 oracle, "
                      f"1 thread of {ncpu} on '{model}')"}


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
    ap.add_argument("--nx", type=int, default=512, help="cells along x")
    ap.add_argument("--ny", type=int, default=512, help="cells along y")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MB",
                    help="instead: time a plain device copy of MB megabytes (counter calibration)")
    ap.add_argument("--prec", default="f64", choices=["f64", "f32", "mixed"])
    ap.add_argument("--weno", default="prim", choices=["prim", "char"],
                    help="WENO5 on primitive (default) or characteristic variables (FP64)")
    ap.add_argument("--graph", action="store_true", help="replay the timed steps from a HIP graph")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle time")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint:forward cost measurement")
    ap.add_argument("--workload", default="quadrant", choices=["quadrant", "cylinder", "sod", "paper-cylinder"],
                    help="quadrant: the four-quadrant Riemann problem (default); cylinder: the viscous "
                         "shock-cylinder case at 1024x512; sod: the 200-cell shock tube (each prints its "
                         "own line)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(the path would shard by spatial slabs with a 3-cell halo exchange per stage)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2601_04400_amd import Grid, inputs

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

    if args.workload == "cylinder":
        print(json.dumps(cylinder_workload(args)), flush=True)
        return
    if args.workload == "sod":
        print(json.dumps(sod_workload(args)), flush=True)
        return
    if args.workload == "paper-cylinder":
        print(json.dumps(paper_cylinder_workload(args)), flush=True)
        return

    nx, ny, K, W = args.nx, args.ny, args.steps, args.warmup
    n2 = nx * ny
    char = args.weno == "char"
    g = Grid(nx, ny, prec=args.prec, weno_char=char)
    U = g.prim_to_cons(torch.from_numpy(inputs.riemann2d_prim(nx, ny)))
    g.set_time(0.0, 1e30)  # no end time inside the run: every step is a full step
    for _ in range(W):
        g.step(U)
    torch.cuda.synchronize()

    graph = None
    if args.graph:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            g.step(U)
        torch.cuda.current_stream().wait_stream(s)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            for _ in range(K):
                g.step(U)
        torch.cuda.synchronize()

    # pass A: the measurement (wall clock, and HIP events on the stream the
    # stage kernels run on: torch's current stream, which the grid adopts)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    if graph is not None:
        graph.replay()
    else:
        for _ in range(K):
            g.step(U)
    ev1.record()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = el * 1e3 / K
    value = n2 * K / el

    # pass B: the same K steps with HIP events around every kernel
    g.profile(True)
    for _ in range(K):
        g.step(U)
    prof = g.profile_read()
    g.profile(False)
    flags, fb = g.poll_faults()

    esize = 8 if args.prec == "f64" else 4
    # average stage-kernel launch: the timed region holds exactly 3 K stage
    # launches and nothing else (the automatic step is fused into them)
    launch_s = gpu_ms * 1e-3 / (3 * K)
    bytes_launch = WORDS_PER_CELL_STEP * esize * n2 / 3
    gbs = bytes_launch / launch_s / 1e9
    flops_cell = FLOPS_PER_CELL_STAGE_CHAR if char else FLOPS_PER_CELL_STAGE
    tflops = flops_cell * n2 / launch_s / 1e12
    fpeak = FP64_PEAK_TFLOPS if args.prec in ("f64", "mixed") else FP32_PEAK_TFLOPS
    traffic = None
    if (not char and MEASURED_TRAFFIC["workload"] == (nx, ny, args.prec)
            and MEASURED_TRAFFIC["sources_sha256"] == stage_sources_sha256()):
        traffic = MEASURED_TRAFFIC["bytes_per_launch"]
    hbm = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic}
    alu = {"bound": "alu", "achieved": round(tflops, 2), "peak": fpeak, "unit": "TFLOP/s",
           "frac": round(tflops / fpeak, 4), "traffic": traffic}
    roof = alu if alu["frac"] >= hbm["frac"] else hbm
    roof = dict(roof)
    roof["kernel"] = "stage_kernel (3 launches per step)"
    roof["stage_us_per_launch"] = round(launch_s * 1e6, 3)
    roof["launches_timed"] = 3 * K
    roof["algorithmic_bytes_per_launch"] = bytes_launch
    roof["algorithmic_flops_per_launch"] = flops_cell * n2
    roof["other_bound"] = hbm if roof["bound"] == "alu" else alu

    out = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.prec, "data": "synthetic",
        "config": {"workload": f"2D Euler four-quadrant Riemann problem {nx}x{ny} on [0,1]^2, gamma 1.4, "
                               "seeded +-5% quadrant states, transmissive, "
                               + ("characteristic-wise " if char else "") + "WENO5-JS+HLLC, SSP-RK3, CFL 0.5",
                   "nx": nx, "ny": ny, "prec": args.prec, "graph": bool(args.graph), "weno": args.weno},
        "hbm_frac_of_peak": round(WORDS_PER_CELL_STEP * esize * n2 * K / el / 1e9 / HBM_PEAK_GBS, 4),
        "hbm_copy_ceiling_GBs": copy_ceiling(),
        "roofline": roof,
        # per-launch times with an event pair around every launch (second
        # pass; includes each pair's own overhead of about a microsecond)
        "kernel_ms_event_bracketed": {k: round(v[0] / max(v[1], 1), 5) for k, v in prof.items() if v[1]},
        "faults": {"flags": flags, "fallback_faces": fb},
    }
    if not args.no_adjoint:
        out["adjoint"] = adjoint_ratio()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(nx, ny, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
