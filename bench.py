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
    pass (segment replays included) over the forward pass."""
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
    res = {}
    for rep in range(2):  # second repetition is the measurement
        U0.grad = None
        U0.requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        U = rollout(g, U0, params, steps, dt, every)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        U.backward(torch.ones_like(U))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        res = {"forward_ms": round((t1 - t0) * 1e3, 3), "backward_ms": round((t2 - t1) * 1e3, 3),
               "ratio": round((t2 - t1) / (t1 - t0), 3)}
    res["workload"] = (f"inviscid Mach-3 shock on a cylinder, {n}x{n}, {steps} fixed RK3 steps, "
                       f"checkpoint every {every}, slip immersed boundary; backward includes segment replays")
    return res


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
    ap.add_argument("--graph", action="store_true", help="replay the timed steps from a HIP graph")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle time")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint:forward cost measurement")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the path would shard by spatial slabs with halo exchange, see the design notes)",
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

    nx, ny, K, W = args.nx, args.ny, args.steps, args.warmup
    n2 = nx * ny
    g = Grid(nx, ny, prec=args.prec)
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

    # pass A: the measurement
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if graph is not None:
        graph.replay()
    else:
        for _ in range(K):
            g.step(U)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
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
    stage_ms = sum(prof[k][0] for k in ("stage1", "stage2", "stage3")) / K
    launches = sum(prof[k][1] for k in ("stage1", "stage2", "stage3"))
    bytes_step = WORDS_PER_CELL_STEP * esize * n2
    gbs = bytes_step / (stage_ms * 1e-3) / 1e9
    tflops = 3 * FLOPS_PER_CELL_STAGE * n2 / (stage_ms * 1e-3) / 1e12
    fpeak = FP64_PEAK_TFLOPS if args.prec in ("f64", "mixed") else FP32_PEAK_TFLOPS
    hbm = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None}
    alu = {"bound": "alu", "achieved": round(tflops, 2), "peak": fpeak, "unit": "TFLOP/s",
           "frac": round(tflops / fpeak, 4), "traffic": None}
    roof = alu if alu["frac"] >= hbm["frac"] else hbm
    roof = dict(roof)
    roof["kernel"] = "stage_kernel (3 launches per step)"
    roof["stage_us_per_launch"] = round(stage_ms * 1e3 / 3, 3)
    roof["launches_timed"] = launches
    roof["other_bound"] = hbm if roof["bound"] == "alu" else alu

    out = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.prec, "data": "synthetic",
        "config": {"workload": f"2D Euler four-quadrant Riemann problem {nx}x{ny} on [0,1]^2, gamma 1.4, "
                               "seeded +-5% quadrant states, transmissive, WENO5-JS+HLLC, SSP-RK3, CFL 0.5",
                   "nx": nx, "ny": ny, "prec": args.prec, "graph": bool(args.graph)},
        "hbm_frac_of_peak": round(bytes_step * K / el / 1e9 / HBM_PEAK_GBS, 4),
        "roofline": roof,
        "kernel_ms": {k: round(v[0] / max(v[1], 1), 5) for k, v in prof.items() if v[1]},
        "faults": {"flags": flags, "fallback_faces": fb},
    }
    if not args.no_adjoint:
        out["adjoint"] = adjoint_ratio()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(nx, ny, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
