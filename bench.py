"""Benchmark: MGRIT solves of periodic linear advection on one MI355X.

One step = one complete MGRIT solve, to a 1e-10 relative residual, of the
workload 'advection1d-4096x4096-erk3u3-vcycle-m8': u_t + u_x = 0 on [-1, 1),
nx = nt = 4096, CFL 0.85, third-order upwind + three-stage ERK3, V-cycle with
m = 8 down to 8 coarse steps (4096 -> 512 -> 64 -> 8), FCF relaxation, the
corrected semi-Lagrangian coarse operator, FP64, seeded 16-mode Fourier u0 and
a uniformly random initial iterate.  The timed region starts with the inputs in
HBM and ends with the whole space-time solution [nt+1][nx] written to HBM.

Printed as one JSON line: space-time DOF/s (nx*nt per solve), p50/p99 solve
latency, the sequential GPU time-stepping baseline, the roofline of the
dominant kernel (timed live with HIP events on the library's stream) and the
oracle timed on host cores on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

NX = NT = 4096
CFL = 0.85
P = Q = 3
MS = [8, 8, 8]
SEED = 1002
WORKLOAD = "advection1d-4096x4096-erk3u3-vcycle-m8"

COPY_BYTES = 1 << 30

FP64_VALU_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


def kernel_source_hash():
    """Hash of every library source (kernels, launch shapes, host driver)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2209_06916_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def phi_flops_per_dof():
    """Algorithmic flops per point per fine step (one FMA = 2 flops): ERK3 as
    three products with the 4-tap U3 stencil plus one axpy each."""
    taps = P + 1
    stages = 3
    return 2 * stages * (taps + 1)


def cpu_baseline(u0, v0):
    """The oracle, unmodified, timed on one host core on the same workload: one
    complete V-cycle solve to 1e-10 (nx = nt = 4096, hierarchy 4096 -> 512 ->
    64 -> 8), several seconds of CPU work."""
    from oracle import mgrit as omg
    from threadpoolctl import threadpool_limits
    nt_s = NT
    H = omg.Hierarchy(NX, nt_s, P, "erk", Q, CFL, MS)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        _, info = omg.solve(H, u0, v0[: nt_s + 1], rtol=1e-10, max_iter=30)
        dt = time.perf_counter() - t0
    return dict(value=NX * nt_s / dt, unit="DOF/s", cores=1, kind="oracle",
                sample=f"one oracle V-cycle MGRIT solve to 1e-10 of the whole workload (nx={NX}, nt={nt_s}, "
                       f"m=8, {info['iterations']} iterations, {dt:.1f} s)")


def phase_work(iterations):
    """Algorithmic (flops, bytes) per solve of each profiled phase.

    Fine relaxation: 2 launches per iteration + 1 (the last pre-relaxation),
    each nt fine steps of nx points (flops), reading and writing one nx-vector
    per CF-interval (bytes; F-points stay on chip).  Coarse levels: every
    application of Psi_l (semi-Lagrangian taps + forward/backward recurrences
    of order (p+1)/2) reads one right-hand-side vector.  Final: nt - nt/m fine
    steps, reads the C-points, writes all nt+1 rows."""
    nc0 = NT // MS[0]
    fine_launches = 2 * (iterations + 1)
    fine = (fine_launches * NT * NX * phi_flops_per_dof(), fine_launches * 2 * nc0 * NX * 8, fine_launches)
    k = (P + 1) // 2
    psi_flops = 2 * ((P + 1) + 2 * (2 * k + 1) + 1)
    apps = 0
    launches = 0
    nt_l = NT
    for lev, m in enumerate(MS):
        nt_l //= m
        if lev < len(MS) - 1:
            m_next = MS[lev + 1]
            apps += 2 * nt_l + (nt_l - nt_l // m_next)
            launches += 3
        else:
            apps += nt_l
            launches += 1
    coarse = (iterations * apps * NX * psi_flops, iterations * apps * NX * 8, iterations * launches)
    final = ((NT - nc0) * NX * phi_flops_per_dof(), ((NT + 1) + (nc0 + 1)) * NX * 8, 1)
    return {"fine_relax": fine, "coarse": coarse, "final": final}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="for hardware-counter runs: a few solves plus one elementwise copy of "
                         "COPY_BYTES read + COPY_BYTES written (the counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (the path is a single-GPU build); "
                                   f"--gpus {args.gpus} is not supported"}))
        sys.exit(2)

    import torch
    from paper_2209_06916_amd import inputs, mgrit

    dev = torch.device("cuda:0")
    u0 = inputs.u0_fourier(NX, SEED)
    v0 = inputs.initial_iterate(NT, NX, u0, SEED)
    u0_d = torch.from_numpy(u0).to(dev)
    v0_d = torch.from_numpy(v0).to(dev)
    out = torch.empty((NT + 1, NX), dtype=torch.float64, device=dev)
    prob = mgrit.make_problem(NX, NT, CFL, P, "erk", Q)
    opts = mgrit.make_options(MS, max_levels=len(MS) + 1, rtol=1e-10, max_iter=30)
    solver = mgrit.Solver(prob, opts)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        solver.solve(u0_d, v0_d, u_out=out)
    torch.cuda.synchronize()
    if args.traffic_probe:
        for _ in range(args.steps):
            solver.solve(u0_d, v0_d, u_out=out)
        x = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"traffic_probe": True, "copy_bytes": COPY_BYTES, "solves": args.steps}), flush=True)
        return

    solver.profile_enable(["fine_relax", "coarse", "final"])
    solver.profile_read(reset=True)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    iters = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        info = solver.solve(u0_d, v0_d, u_out=out)
        ends[k].record(stream)
        iters.append(info["iterations"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = solver.profile_read(reset=True)
    solver.profile_enable([])
    lat_ms = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])

    # sequential GPU time-stepping baseline (same u0, same Phi)
    seq_out = torch.empty_like(out)
    solver.sequential(u0_d, seq_out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nseq = 3
    for _ in range(nseq):
        solver.sequential(u0_d, seq_out)
    torch.cuda.synchronize()
    seq_s = (time.perf_counter() - t1) / nseq

    dof = NX * NT
    value = dof * args.steps / wall
    ms_per_step = 1e3 * wall / args.steps

    # dominant kernel by GPU time among the profiled phases
    dom = max(prof, key=lambda k: prof[k]["total_ms"])
    it = int(np.median(iters))
    # Work per solve over kernel time per solve.  The coarse phase also counts
    # the launches of the last iteration's correction, queued before the
    # stopping test is known and returning at once: they add time, no work.
    flops_s, bytes_s, launches_s = phase_work(it)[dom]
    launches = prof[dom]["launches"] / args.steps
    assert launches >= launches_s, (dom, launches, launches_s)
    avg_s = prof[dom]["total_ms"] / prof[dom]["launches"] / 1e3
    flops = flops_s / launches
    bytes_ = bytes_s / launches
    kernel = {"fine_relax": "tile_kernel<8, 2, 1>: level-0 F/C relaxation and C-point residual",
              "coarse": "slc_kernel<4, 2, 4>: coarse-level passes (SL step + periodic banded solve)",
              "final": "tile_kernel<8, 2, 1>: final F-relaxation writing the space-time solution"}[dom]
    ai = flops / bytes_
    ridge = FP64_VALU_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    if ai >= ridge:
        achieved = flops / avg_s / 1e12
        roof = dict(bound="alu", achieved=achieved, peak=FP64_VALU_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=achieved / FP64_VALU_PEAK_TFLOPS)
    else:
        achieved = bytes_ / avg_s / 1e9
        roof = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS)
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tfile):
        with open(tfile) as fh:
            t = json.load(fh)
        if t.get("source_hash") == kernel_source_hash() and t.get("phase") == dom and t.get("workload") == WORKLOAD:
            traffic = t.get("bytes_per_launch")
    roof["traffic"] = traffic
    roof["kernel"] = kernel
    roof["phase"] = dom
    roof["avg_launch_us"] = avg_s * 1e6
    roof["launches_per_solve"] = launches
    roof["working_launches_per_solve"] = launches_s
    roof["algorithmic_flops_per_launch"] = flops
    roof["algorithmic_bytes_per_launch"] = bytes_

    line = {
        "metric": "space-time DOF/s to 1e-10 residual vs seq. stepping; p50/p99 solve latency",
        "value": value,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "nx": NX, "nt": NT, "cfl": CFL, "scheme": "ERK3+U3",
                   "hierarchy": [NT, NT // 8, NT // 64, NT // 512], "relaxation": "FCF",
                   "coarse_operator": "semi-Lagrangian + implicit truncation correction", "rtol": 1e-10},
        "iterations": int(np.median(iters)),
        "latency_ms_p50": float(np.percentile(lat_ms, 50)),
        "latency_ms_p99": float(np.percentile(lat_ms, 99)),
        "sequential_gpu_dof_per_s": dof / seq_s,
        "sequential_gpu_ms": seq_s * 1e3,
        "speedup_vs_sequential": (dof / seq_s) and value / (dof / seq_s),
        "phase_ms_per_solve": {k: v["total_ms"] / args.steps for k, v in prof.items() if v["launches"]},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(u0, v0)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
