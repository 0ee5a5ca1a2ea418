"""Benchmark: MGRIT solves of periodic linear advection on one MI355X.

One step = one complete MGRIT solve, to a 1e-10 relative residual, of the
workload 'advection1d-16384x16384-sdirk3u5-vcycle-m16': u_t + u_x = 0 on
[-1, 1), nx = nt = 16384, CFL 0.5, fifth-order upwind + three-stage SDIRK3
(a periodic banded solve per stage), V-cycle with m = 16
(16384 -> 1024 -> 64 -> 4), FCF relaxation, the corrected semi-Lagrangian
coarse operator, FP64, seeded 16-mode Fourier u0 and a uniformly random
initial iterate (seed 1003).  The timed region starts with the inputs in HBM
and ends with the whole space-time solution [nt+1][nx] written to HBM.

Printed as one JSON line: space-time DOF/s (nx*nt per solve), p50/p99 solve
latency, the sequential GPU time-stepping baseline, the roofline of the
dominant kernel (timed live with HIP events on the library's stream), the
oracle timed on host cores on a bounded sample, and the same solve in mixed
precision and the 4096 x 4096 ERK3 + U3 workload as extra keys.
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

# The workloads (seeded synthetic inputs; the paper uses no dataset).
WORKLOADS = {
    "config3": dict(name="advection1d-16384x16384-sdirk3u5-vcycle-m16", nx=16384, nt=16384, cfl=0.5, p=5,
                    kind="sdirk", q=3, ms=[16, 16, 16], seed=1003, scheme="SDIRK3+U5"),
    "config2": dict(name="advection1d-4096x4096-erk3u3-vcycle-m8", nx=4096, nt=4096, cfl=0.85, p=3, kind="erk",
                    q=3, ms=[8, 8, 8], seed=1002, scheme="ERK3+U3"),
}
HEADLINE = WORKLOADS["config3"]
WORKLOAD = HEADLINE["name"]

COPY_BYTES = 1 << 30

FP64_VALU_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


def kernel_source_hash():
    """Hash of the device-code sources (every .hip and .h of the library)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2209_06916_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def phi_flops_per_dof(wl):
    """Algorithmic flops per point per fine step (one FMA = 2 flops), in the
    form the level-0 kernels evaluate.  ERK3 + U3: R(Z) written out as one
    stencil of s (l + r) + 1 = 10 taps.  SDIRK: R as a polynomial of degree s
    in W = (I + gamma c L_p)^{-1}, each W one causal recurrence of order
    (p+1)/2 and one anti-causal of order (p-1)/2 (1/C folded into the
    coefficients), plus one Horner term per power: s (p + 1) for U5 + SDIRK3,
    18 FMAs.  (The Butcher stage form of SDIRK3 + U5, with an explicit U5
    product and a banded LU solve per stage, counts about 116 flops; the
    windowed kernel executes each recurrence twice, 66 flops.)"""
    stages = 3
    if wl["kind"] == "erk":
        left, right = (wl["p"] + 1) // 2, (wl["p"] - 1) // 2
        return 2 * (stages * (left + right) + 1)
    kf, kb = (wl["p"] + 1) // 2, (wl["p"] - 1) // 2
    return 2 * (stages * (kf + kb) + stages)


def psi_flops_per_dof(wl):
    """Algorithmic flops per point of one coarse step Psi = T^{-1} S: p+1
    interpolation taps, then the causal and anti-causal recurrences of order
    k = (p+1)/2 each and the scale by 1/C."""
    k = (wl["p"] + 1) // 2
    return 2 * ((wl["p"] + 1) + 2 * k + 1)


def cpu_baseline(wl):
    """The oracle, unmodified, timed on one host core on a bounded sample of
    the workload: a complete V-cycle MGRIT solve to 1e-10 of its first 512
    time steps (nx = 16384, m = 16, 512 -> 32 -> 2; 10-40 s of CPU work).
    The whole 16384 x 16384 solve takes the oracle about 48 minutes."""
    from oracle import mgrit as omg
    from paper_2209_06916_amd import inputs
    from threadpoolctl import threadpool_limits
    nx, nt_s, ms = wl["nx"], 512, [16, 16]
    u0 = inputs.u0_fourier(nx, wl["seed"])
    v0 = inputs.initial_iterate(nt_s, nx, u0, wl["seed"])
    H = omg.Hierarchy(nx, nt_s, wl["p"], wl["kind"], wl["q"], wl["cfl"], ms)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        _, info = omg.solve(H, u0, v0, rtol=1e-10, max_iter=30)
        dt = time.perf_counter() - t0
    return dict(value=nx * nt_s / dt, unit="DOF/s", cores=1, kind="oracle",
                sample=f"one oracle V-cycle MGRIT solve to 1e-10 of the first {nt_s} time steps of the workload "
                       f"(nx={nx}, m=16, levels {nt_s} -> {nt_s // 16} -> 1, {info['iterations']} iterations, "
                       f"{dt:.1f} s on one core)")


def phase_work(wl, iterations):
    """Algorithmic (flops, bytes, working launches) per solve of each profiled phase.

    Rows are nx doubles.  Level 0 (nc0 = nt/m intervals): pass A reads C_k and
    writes C'_{k+1} (2 nc0 rows), pass B reads C'_k and C'_{k+1} and writes r
    (3 nc0 rows); F-points never leave the chip; each pass takes nt fine steps.
    Coarse level l (nt_l points, nc_l intervals): pass A 2 nc_l + nt_l rows (the
    right-hand side row of every step), pass B 3 nc_l + nt_l, post-F relaxation
    nc_l C-rows, (m_l - 1) nc_l right-hand sides and a read-modify-write of every
    parent row (2 nt_l); the coarsest sweep nt_L right-hand sides and 2 nt_L
    parent rows.  Every Psi application: semi-Lagrangian taps and the forward and
    backward recurrences of order (p+1)/2.  Final pass: nt - nc0 fine steps,
    reads the C-points and writes all nt+1 rows."""
    NX, NT, MS = wl["nx"], wl["nt"], wl["ms"]
    row = NX * 8
    nc0 = NT // MS[0]
    passes = iterations + 1  # pre-relaxation of every iteration and of the last check
    fine = (2 * passes * NT * NX * phi_flops_per_dof(wl), passes * (2 + 3) * nc0 * row, 2 * passes)
    psi_flops = psi_flops_per_dof(wl)
    apps = rows = launches = 0
    nt_l = NT
    for lev, m in enumerate(MS):
        nt_l //= m  # points of level lev+1
        if lev < len(MS) - 1:
            nc = nt_l // MS[lev + 1]
            apps += 2 * nt_l + (nt_l - nc)
            rows += (2 * nc + nt_l) + (3 * nc + nt_l) + (nc + (nt_l - nc) + 2 * nt_l)
            launches += 3
        else:
            apps += nt_l
            rows += nt_l + 2 * nt_l
            launches += 1
    coarse = (iterations * apps * NX * psi_flops, iterations * rows * row, iterations * launches)
    final = ((NT - nc0) * NX * phi_flops_per_dof(wl), ((NT + 1) + (nc0 + 1)) * row, 1)
    return {"fine_relax": fine, "coarse": coarse, "final": final}


PROFILE_COMMANDS = {
    "trace": "rocprofv3 --kernel-trace --stats --output-format csv -d <dir>/trace -o run -- "
             "python3 bench.py --steps 10 --warmup 2 --no-cpu-baseline --no-extras",
    "fetch": "rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir>/fetch -o run -- "
             "python3 bench.py --steps 2 --warmup 1 --traffic-probe",
    "write": "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir>/write -o run -- "
             "python3 bench.py --steps 2 --warmup 1 --traffic-probe",
    "serve": "rocprofv3 --kernel-trace --stats --output-format csv -d <dir>/serve -o run -- "
             "python3 bench.py --serve 512 --no-extras",
    "sq": "rocprofv3 --pmc SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_INSTS_VALU "
          "SQ_ACTIVE_INST_VALU SQ_INSTS_LDS --output-format csv -d <dir>/sq -o run -- "
          "python3 bench.py --steps 1 --warmup 0 --traffic-probe",
    "sq2": "rocprofv3 --pmc SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_INSTS_VALU "
           "SQ_ACTIVE_INST_VALU SQ_INSTS_LDS --output-format csv -d <dir>/sq2 -o run -- "
           "python3 bench.py --steps 1 --warmup 0 --traffic-probe --probe-workload config2",
}
SQ_COUNTERS = ["SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_INSTS_VALU",
               "SQ_ACTIVE_INST_VALU", "SQ_INSTS_LDS"]
SERVE_WORKLOAD = "served-advection1d-512-requests"


def _short(name):
    name = name.replace("void ", "").replace("mgrit::(anonymous namespace)::", "")
    return name.split("(")[0]


def _write_sq_summary(sq_csv, prof_dir, wl_name, what, command):
    """profiles/counters_<workload>.txt from one rocprofv3 --pmc run of the SQ counters."""
    import csv
    per = {}
    for r in csv.DictReader(open(sq_csv)):
        k = _short(r["Kernel_Name"])
        if k.startswith("at::") or k.startswith("__amd"):
            continue
        key = (r.get("Dispatch_Id") or r.get("Correlation_Id"), r["Counter_Name"])
        per.setdefault(k, {}).setdefault(r["Counter_Name"], {})
        per[k][r["Counter_Name"]][key[0]] = per[k][r["Counter_Name"]].get(key[0], 0.0) + float(r["Counter_Value"])
    lines = [f"# rocprofv3 SQ counters -- workload {wl_name}",
             f"# ({what}, no warm-up; values summed over the device per dispatch, then averaged over",
             "# dispatches; wave-cycle counters as the hardware counts them)",
             "# command (repository root on the GPU box, after cd /tmp && export TMPDIR=/tmp):",
             "#   " + command,
             "#", "# kernel: dispatches; " + ", ".join(SQ_COUNTERS) + " (per dispatch)",
             "#   derived: VALU and LDS instructions per wavefront; WAIT_ANY / WAVE_CYCLES (any wait);",
             "#   WAIT_INST_ANY / WAVE_CYCLES (dependency waits); ACTIVE_INST_VALU / WAVE_CYCLES (VALU issue)"]
    for k, cs in sorted(per.items()):
        avg = {c: float(np.mean(list(cs[c].values()))) for c in SQ_COUNTERS if c in cs}
        nd = max(len(v) for v in cs.values())
        lines.append(f"  {k}: {nd} dispatches; " + ", ".join(f"{avg.get(c, float('nan')):.4g}" for c in SQ_COUNTERS))
        w = avg.get("SQ_WAVES", 0.0)
        wc = avg.get("SQ_WAVE_CYCLES", 0.0)
        if w > 0 and wc > 0:
            lines.append(f"    VALU/wave {avg.get('SQ_INSTS_VALU', 0.0) / w:.0f}, LDS/wave "
                         f"{avg.get('SQ_INSTS_LDS', 0.0) / w:.0f}, any wait "
                         f"{avg.get('SQ_WAIT_ANY', 0.0) / wc:.2f}, dependency waits "
                         f"{avg.get('SQ_WAIT_INST_ANY', 0.0) / wc:.2f}, VALU issue "
                         f"{avg.get('SQ_ACTIVE_INST_VALU', 0.0) / wc:.2f} of wave-cycles")
    with open(os.path.join(prof_dir, f"counters_{wl_name}.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


def summarize_profiles(d):
    """Turn the three rocprofv3 runs under directory d (made by PROFILE_COMMANDS,
    run from the repository root after `cd /tmp && export TMPDIR=/tmp`) into
    profiles/kernel_stats_<workload>.txt, profiles/traffic_<workload>.txt and
    profiles/traffic.json (the counters scaled by what they read for the
    probe's 1 GiB elementwise copy)."""
    import csv
    prof_dir = os.path.join(ROOT, "profiles")
    trace_csv = os.path.join(d, "trace", "run_kernel_stats.csv")
    if os.path.exists(trace_csv):
        rows = list(csv.DictReader(open(trace_csv)))
        tot = sum(float(r["TotalDurationNs"]) for r in rows)
        lines = [f"# rocprofv3 kernel statistics -- workload {WORKLOAD}",
                 "# (MGRIT solves: 2 warm-up, 3 with every phase timed by events, 10 timed; then 4 runs of sequential",
                 "# time-stepping of the same problem; then 4 MGRIT solves without the final F-pass)",
                 "# command (repository root on the GPU box, after cd /tmp && export TMPDIR=/tmp):",
                 "#   " + PROFILE_COMMANDS["trace"].replace("<dir>", "gpurun_out/prof"),
                 "#", f"# {'kernel':52s} {'calls':>6s} {'avg_us':>10s} {'total_ms':>10s} {'share':>7s}"]
        for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
            lines.append(f"  {_short(r['Name']):52s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.2f} "
                         f"{float(r['TotalDurationNs']) / 1e6:10.3f} {100 * float(r['TotalDurationNs']) / tot:6.2f}%")
        trace_csv = os.path.join(d, "trace", "run_kernel_trace.csv")
        if os.path.exists(trace_csv):
            # the same kernel runs several launch shapes (relaxation passes,
            # sequential stepping): durations per shape, from the kernel trace
            shapes = {}
            for r in csv.DictReader(open(trace_csv)):
                k = _short(r["Kernel_Name"])
                if not k.startswith("wstep_kernel"):
                    continue
                wgs = int(r["Grid_Size_X"]) // max(1, int(r["Workgroup_Size_X"]))
                shapes.setdefault((k, wgs), []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
            lines += ["#", "# per launch shape (kernel trace; workgroups per launch):",
                      f"# {'kernel':44s} {'workgroups':>10s} {'calls':>6s} {'avg_us':>10s} {'median_us':>10s}"]
            for (k, wgs), ds in sorted(shapes.items(), key=lambda kv: -sum(kv[1])):
                lines.append(f"  {k:44s} {wgs:10d} {len(ds):6d} {float(np.mean(ds)):10.2f} {float(np.median(ds)):10.2f}")
        lines += ["#", "# wstep_kernel<32, 1, 3, 2, 512, double>: SDIRK3 + U5 steps (32 points per thread, 512 threads);",
                  "#   grid 524288: level-0 relaxation passes (1024 intervals) and the final F-pass; grid 512: sequential",
                  "#   time-stepping (one workgroup, 16384 steps)",
                  "# wstep_kernel<32, 2, 3, 3, 512, double>: corrected semi-Lagrangian steps of levels 1-3, one launch per",
                  "#   pass (the last correction of each solve returns at once)",
                  "# solve_ctl_kernel: residual norm + stopping test."]
        with open(os.path.join(prof_dir, f"kernel_stats_{WORKLOAD}.txt"), "w") as fh:
            fh.write("\n".join(lines) + "\n")

    serve_csv = os.path.join(d, "serve", "run_kernel_stats.csv")
    if os.path.exists(serve_csv):
        rows = list(csv.DictReader(open(serve_csv)))
        tot = sum(float(r["TotalDurationNs"]) for r in rows)
        lines = [f"# rocprofv3 kernel statistics -- workload {SERVE_WORKLOAD}",
                 "# (bench.py --serve 512 --no-extras: 2 x 16 warm-up requests, then the float64 512-request stream",
                 "# served with 1 in flight (polling loop), 16 in flight (one host thread per request), 16 in flight",
                 "# (polling loop), then with Poisson arrivals; the mixed-precision stream is not traced; the profiler",
                 "# slows the host loop,",
                 "# so the rates it prints are lower than without it)",
                 "# command (repository root on the GPU box, after cd /tmp && export TMPDIR=/tmp):",
                 "#   " + PROFILE_COMMANDS["serve"].replace("<dir>", "gpurun_out/prof"),
                 f"# total kernel time {tot / 1e6:.1f} ms over {sum(int(r['Calls']) for r in rows)} launches",
                 "#", f"# {'kernel':52s} {'calls':>6s} {'avg_us':>10s} {'total_ms':>10s} {'share':>7s}"]
        for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:25]:
            lines.append(f"  {_short(r['Name']):52s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.2f} "
                         f"{float(r['TotalDurationNs']) / 1e6:10.3f} {100 * float(r['TotalDurationNs']) / tot:6.2f}%")
        with open(os.path.join(prof_dir, f"kernel_stats_{SERVE_WORKLOAD}.txt"), "w") as fh:
            fh.write("\n".join(lines) + "\n")

    for sub, wl_name, what in (("sq", WORKLOAD, "one MGRIT solve"),
                               ("sq2", WORKLOADS["config2"]["name"], "one MGRIT solve of config 2")):
        sq_csv = os.path.join(d, sub, "run_counter_collection.csv")
        if os.path.exists(sq_csv):
            _write_sq_summary(sq_csv, prof_dir, wl_name, what, PROFILE_COMMANDS[sub].replace("<dir>", "gpurun_out/prof"))

    if not (os.path.exists(os.path.join(d, "fetch", "run_counter_collection.csv")) and
            os.path.exists(os.path.join(d, "write", "run_counter_collection.csv"))):
        return
    def counters(sub, name):
        per = {}
        order = []
        for r in csv.DictReader(open(os.path.join(d, sub, "run_counter_collection.csv"))):
            if r["Counter_Name"] != name:
                continue
            k = _short(r["Kernel_Name"])
            per.setdefault(k, []).append(float(r["Counter_Value"]))
            order.append(k)
        return per, order

    fetch, forder = counters("fetch", "FETCH_SIZE")
    write, _ = counters("write", "WRITE_SIZE")
    # the calibration copy is the probe's last dispatch
    copy_name = forder[-1]
    copy_kib = COPY_BYTES / 1024
    fscale = copy_kib / fetch[copy_name][-1]
    wscale = copy_kib / write[copy_name][-1]
    lines = [f"# rocprofv3 HBM traffic counters -- workload {WORKLOAD}",
             "# commands (two separate runs, one counter each; repository root, after cd /tmp && export TMPDIR=/tmp):",
             "#   " + PROFILE_COMMANDS["fetch"].replace("<dir>", "gpurun_out/prof"),
             "#   " + PROFILE_COMMANDS["write"].replace("<dir>", "gpurun_out/prof"),
             f"# calibration: the probe's elementwise copy ({copy_name}) reads and writes {COPY_BYTES >> 20} MiB",
             f"#   FETCH_SIZE read {fetch[copy_name][-1]:.1f} KiB for {copy_kib:.0f} KiB -> scale {fscale:.4f}",
             f"#   WRITE_SIZE read {write[copy_name][-1]:.1f} KiB for {copy_kib:.0f} KiB -> scale {wscale:.4f}",
             "# per dispatch: mean over dispatches (level-0 kernel: median, see below)",
             "#", f"# {'kernel':40s} {'dispatches':>10s} {'FETCH_KiB/disp':>15s} {'WRITE_KiB/disp':>15s} "
                  f"{'scaled_MB/disp':>15s}"]
    # per dispatch: the mean, as the bench averages its launch durations;
    # for the level-0 kernel the median, since it also runs the one final
    # F-pass of each solve, which writes every time point
    result = {}
    for k in fetch:
        if k == copy_name or k not in write or k.startswith("at::"):
            continue
        avg = np.median if k == PHASE_KERNELS["fine_relax"] else np.mean
        fk = float(avg(fetch[k]))
        wk = float(avg(write[k]))
        mb = (fk * fscale + wk * wscale) * 1024 / 1e6
        lines.append(f"  {k:40s} {len(fetch[k]):10d} {fk:15.1f} {wk:15.1f} {mb:15.2f}")
        for ph, kn in PHASE_KERNELS.items():
            if k == kn and ph != "final":
                result[ph] = dict(kernel=k, fetch_kib_per_dispatch=fk, write_kib_per_dispatch=wk,
                                  bytes_per_launch=(fk * fscale + wk * wscale) * 1024)
    lines += ["#", f"# {PHASE_KERNELS['fine_relax']}: level-0 passes and the final F-pass (median: a pass A",
              "#   reads and writes the 1025 C-point rows, 2 x 134 MB); " + PHASE_KERNELS["coarse"] + ":",
              "#   every coarse-level pass of levels 1-3 (mean over the passes of a V-cycle)"]
    with open(os.path.join(prof_dir, f"traffic_{WORKLOAD}.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    if result:
        with open(os.path.join(prof_dir, "traffic.json"), "w") as fh:
            json.dump({"workload": WORKLOAD, "source_hash": kernel_source_hash(), "fetch_scale": fscale,
                       "write_scale": wscale, "phases": result, "source": f"profiles/traffic_{WORKLOAD}.txt"},
                      fh, indent=1)
    print("\n".join(lines))


def _progress(msg):
    print(msg, file=sys.stderr, flush=True)


def serve_bench(n, seed, with_mixed=True):
    """Config 5: n independent 1D solves (nx, nt in 256..8192, ERK1/3/5 with
    the matching upwind order, CFL U(0.5, 0.9), m in {4, 8, 16}, multilevel
    down to <= 8 coarse steps, seeded 16-mode Fourier u0, zero initial
    iterate).  Throughput with one solve in flight and with up to 16 in
    flight (all requests queued at once; one host thread per request in
    flight, and the single-thread polling loop for comparison), then latency
    under Poisson arrivals at 0.8x the single-stream capacity.  with_mixed:
    also serve the stream in mixed precision."""
    from paper_2209_06916_amd import serve
    reqs = serve.synthetic_stream(n, seed=seed, rate_hz=0)
    dof = sum(r.nx * r.nt for r in reqs)
    serve.ThreadedServer(max_inflight=16).run(reqs[:16], realtime=False)  # warm-up (kernels, allocator)
    serve.Server(max_inflight=16).run(reqs[:16], realtime=False)
    t = time.perf_counter()
    one = serve.Server(max_inflight=1).run(reqs, realtime=False)
    t_one = time.perf_counter() - t
    _progress(f"serve: one in flight {t_one:.2f} s")
    t = time.perf_counter()
    many = serve.ThreadedServer(max_inflight=16).run(reqs, realtime=False)
    t_many = time.perf_counter() - t
    _progress(f"serve: 16 in flight, threaded {t_many:.2f} s")
    t = time.perf_counter()
    serve.Server(max_inflight=16).run(reqs, realtime=False)
    t_loop = time.perf_counter() - t
    _progress(f"serve: 16 in flight, polling {t_loop:.2f} s")
    by1 = {r.tag: r for r in one}
    same = all(np.array_equal(by1[r.tag].u_final, r.u_final) for r in many)
    # the same stream served in mixed precision (zero initial iterate, so the
    # float64 and the full space-time residual start from the same norm)
    mixed, t_mixed, mixed_err = [], float("nan"), float("nan")
    if with_mixed:
        mixed_reqs = serve.synthetic_stream(n, seed=seed, rate_hz=0, precision="mixed")
        serve.ThreadedServer(max_inflight=16).run(mixed_reqs[:16], realtime=False)
        t = time.perf_counter()
        mixed = serve.ThreadedServer(max_inflight=16).run(mixed_reqs, realtime=False)
        t_mixed = time.perf_counter() - t
        _progress(f"serve: mixed precision {t_mixed:.2f} s")
        mixed_err = max(float(np.linalg.norm(r.u_final - by1[r.tag].u_final) / np.linalg.norm(by1[r.tag].u_final))
                        for r in mixed)
    rate = 0.8 * n / t_one
    arrivals = serve.synthetic_stream(n, seed=seed, rate_hz=rate)
    t = time.perf_counter()
    live = serve.ThreadedServer(max_inflight=16).run(arrivals, realtime=True)
    t_live = time.perf_counter() - t
    lat = np.array([r.latency for r in live]) * 1e3
    line = {
        "metric": "served MGRIT solves: space-time DOF/s and p50/p99 request latency",
        "value": dof / t_many,
        "unit": "DOF/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"served-advection1d-{n}-requests", "requests": n, "sizes": "nx, nt in 256..8192",
                   "schemes": "ERK1/3/5 + U1/3/5", "cfl": "U(0.5, 0.9)", "m": [4, 8, 16], "max_inflight": 16,
                   "server": "one host thread per request in flight"},
        "dof_per_s_one_in_flight": dof / t_one,
        "dof_per_s_16_in_flight": dof / t_many,
        "dof_per_s_16_in_flight_polling_loop": dof / t_loop,
        "mixed_dof_per_s_16_in_flight": dof / t_mixed if mixed else None,
        "mixed_all_converged": bool(mixed) and all(r.status == 0 for r in mixed),
        "mixed_max_rel_diff_vs_fp64": mixed_err if mixed else None,
        "concurrency_speedup": t_one / t_many,
        "same_results_alone_and_in_mix": bool(same),
        "all_converged": all(r.status == 0 for r in many),
        "poisson_rate_hz": rate,
        "poisson_dof_per_s": dof / t_live,
        "latency_ms_p50": float(np.percentile(lat, 50)),
        "latency_ms_p99": float(np.percentile(lat, 99)),
    }
    print(json.dumps(line), flush=True)


def precision_bench(steps):
    """Float64 MGRIT against mixed precision (float32 inner MGRIT in float64
    refinement) on config 2 (nx = nt = 4096, ERK3 + U3, c = 0.85, m = 8,
    4 levels) and config 3 (nx = nt = 16384, SDIRK3 + U5, c = 0.5, m = 16,
    levels 16384 -> 1024 -> 64 -> 4), from the seeded U[0,1) initial
    iterate.  Float64 MGRIT stops at a C-point residual of 1e-10 of its
    first one (the bench's criterion); mixed precision measures the full
    space-time residual, whose first value also carries the random
    F-points, so it stops at 1e-12 of it, which gives the same solution
    error.  Each result's error is taken against sequential time-stepping
    on the GPU (mgrit_sequential, the exact solution of the one-step system
    up to rounding).  A last, untimed solve of each records the GPU time of
    its phases with the library's event profiler."""
    import torch
    from paper_2209_06916_amd import inputs, mgrit
    dev = torch.device("cuda:0")
    cases = [("advection1d-4096x4096-erk3u3-vcycle-m8", 4096, 4096, 3, "erk", 3, 0.85, [8, 8, 8], 1002),
             ("advection1d-16384x16384-sdirk3u5-vcycle-m16", 16384, 16384, 5, "sdirk", 3, 0.5, [16, 16, 16], 1003)]
    for name, nx, nt, p, kind, q, c, ms, seed in cases:
        u0 = inputs.u0_fourier(nx, seed)
        v0 = torch.from_numpy(inputs.initial_iterate(nt, nx, u0, seed)).to(dev)
        u0_d = torch.from_numpy(u0).to(dev)
        prob = mgrit.make_problem(nx, nt, c, p, kind, q)
        out = torch.empty((nt + 1, nx), dtype=torch.float64, device=dev)
        ref = torch.empty((nt + 1, nx), dtype=torch.float64, device=dev)
        line = {"workload": name, "dof": nx * nt, "steps": steps}
        seq = mgrit.Solver(prob, mgrit.make_options(ms, max_levels=len(ms) + 1))
        seq.sequential(u0_d, ref)
        torch.cuda.synchronize()
        ref_norm = torch.linalg.vector_norm(ref).item()
        for prec in ("fp64", "mixed"):
            s = mgrit.Solver(prob, mgrit.make_options(ms, max_levels=len(ms) + 1,
                                                      rtol=1e-10 if prec == "fp64" else 1e-12, max_iter=30,
                                                      precision=prec))
            info = s.solve(u0_d, v0, u_out=out)  # warm-up
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(steps):
                info = s.solve(u0_d, v0, u_out=out)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t) / steps
            err = torch.linalg.vector_norm(out - ref).item() / ref_norm
            s.profile_enable(mgrit.PROF_PHASES)
            s.solve(u0_d, v0, u_out=out)
            prof = s.profile_read()
            line[prec] = {"ms_per_solve": 1e3 * wall, "dof_per_s": nx * nt / wall, "status": info["status"],
                          "iterations": info["iterations"], "inner_iterations": info["inner_iterations"],
                          "rel_l2_error_vs_sequential": err,
                          "phase_ms": {k: round(v["total_ms"], 3) for k, v in prof.items() if v["launches"]}}
            s.close()
        line["mixed_speedup"] = line["fp64"]["ms_per_solve"] / line["mixed"]["ms_per_solve"]
        print(json.dumps(line), flush=True)
        seq.close()
        del out, ref, v0
        torch.cuda.empty_cache()


def gmres_bench(steps):
    """Exact against GMRES coarse solves (Sec. 6.3: zero start, 1e-2 relative
    residual, at most 20 iterations) on the Table 3 grid (256 x 1024,
    ERK3+U3 at 0.85 c_max, m = 8), config 2 and config 3, each from the
    seeded U[0,1) initial iterate: wall time per solve, iterations, and the
    coarse levels' GPU time from the library's event profiler."""
    import torch
    from paper_2209_06916_amd import inputs, mgrit
    dev = torch.device("cuda:0")
    cases = [("advection1d-256x1024-erk3u3-vcycle-m8", 256, 1024, 0.85 * 1.6258907, 3, "erk", 3, [8, 8, 8], 1002),
             ("advection1d-4096x4096-erk3u3-vcycle-m8", 4096, 4096, 0.85, 3, "erk", 3, [8, 8, 8], 1002),
             ("advection1d-16384x16384-sdirk3u5-vcycle-m16", 16384, 16384, 0.5, 5, "sdirk", 3, [16, 16, 16], 1003)]
    for name, nx, nt, c, p, kind, q, ms, seed in cases:
        line = {"workload": name}
        u0 = torch.from_numpy(inputs.u0_fourier(nx, seed)).to(dev)
        out = torch.empty((nt + 1, nx), dtype=torch.float64, device=dev)
        for key, gm in (("exact", None), ("gmres", (1e-2, 20))):
            s = mgrit.Solver(mgrit.make_problem(nx, nt, c, p, kind, q),
                             mgrit.make_options(ms, max_levels=len(ms) + 1, init_seed=seed, gmres=gm))
            info = s.solve(u0, None, u_out=out)  # warm-up
            n = 1 if (gm and nx >= 16384) else steps
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(n):
                info = s.solve(u0, None, u_out=out)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t) / n
            s.profile_enable(["coarse"])
            s.solve(u0, None, u_out=out)
            coarse = s.profile_read()["coarse"]["total_ms"]
            line[key] = {"ms_per_solve": 1e3 * wall, "iterations": info["iterations"], "coarse_ms": coarse}
            s.close()
        line["gmres_cost"] = line["gmres"]["ms_per_solve"] / line["exact"]["ms_per_solve"]
        print(json.dumps(line), flush=True)
        del out
        torch.cuda.empty_cache()


def twod_bench(steps):
    """Config 4: u_t + a.grad u = 0 on [-1, 1)^2, a = (0.85, 1.0),
    nx = ny = nt = 1024, dt = h/2 (c = (0.425, 0.5)), ERK3 + U3, m = 8,
    3 levels (1024 -> 128 -> 16), u0 = 8 seeded Gaussian bumps of width
    0.1, seeded U[0,1) initial iterate; float64 MGRIT to a C-point residual
    of 1e-10 of its first one, and mixed precision (float32 inner cycles,
    float64 refinement) to a full space-time residual of 1e-12 of its first
    one (it also carries the random F-points); both against sequential
    time-stepping of the same fine step on the GPU."""
    import torch
    from paper_2209_06916_amd import inputs, mgrit
    dev = torch.device("cuda:0")
    n, nt, ms, seed = 1024, 1024, [8, 8], 1004
    u0 = inputs.u0_bumps_2d(n, n, 8, 0.1, seed)
    rng = np.random.default_rng(seed)
    v0 = torch.empty((nt + 1, n, n), dtype=torch.float64, device=dev)
    for k in range(0, nt + 1, 64):  # seeded U[0,1) rows, drawn in blocks
        rows = min(64, nt + 1 - k)
        v0[k:k + rows] = torch.from_numpy(rng.random((rows, n, n))).to(dev)
    u0_d = torch.from_numpy(u0).to(dev)
    v0[0] = u0_d
    pr = mgrit.make_problem_2d(n, n, nt, 0.5, 3)
    out = torch.empty((nt + 1, n, n), dtype=torch.float64, device=dev)
    res = {}
    for prec in ("fp64", "mixed"):
        s = mgrit.Solver2D(pr, mgrit.make_options(ms, max_levels=3, rtol=1e-10 if prec == "fp64" else 1e-12,
                                                  max_iter=30, precision=prec))
        info = s.solve(u0_d, v0, u_out=out)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            info = s.solve(u0_d, v0, u_out=out)
        torch.cuda.synchronize()
        res[prec] = ((time.perf_counter() - t) / steps, info, out.clone() if prec == "fp64" else None)
        if prec == "mixed":
            res[prec] = (res[prec][0], info, None)
            err_mixed_out = out
        s.close()
    del v0
    ref = torch.empty_like(out)
    s = mgrit.Solver2D(pr, mgrit.make_options(ms, max_levels=3))
    s.sequential(u0_d, ref)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        s.sequential(u0_d, ref)
    torch.cuda.synchronize()
    seq = (time.perf_counter() - t) / steps
    rn = torch.linalg.vector_norm(ref)
    err64 = (torch.linalg.vector_norm(res["fp64"][2] - ref) / rn).item()
    err32 = (torch.linalg.vector_norm(err_mixed_out - ref) / rn).item()
    dof = n * n * nt
    w64, i64, _ = res["fp64"]
    w32, i32, _ = res["mixed"]
    print(json.dumps({"workload": "advection2d-1024x1024x1024-erk3u3-vcycle-m8", "dof": dof, "steps": steps,
                      "mgrit_ms": 1e3 * w64, "mgrit_dof_per_s": dof / w64, "iterations": i64["iterations"],
                      "rel_l2_error_vs_sequential": err64,
                      "mixed_ms": 1e3 * w32, "mixed_dof_per_s": dof / w32, "mixed_outer_iterations": i32["iterations"],
                      "mixed_inner_iterations": i32["inner_iterations"], "mixed_rel_l2_error_vs_sequential": err32,
                      "sequential_ms": 1e3 * seq, "sequential_dof_per_s": dof / seq,
                      "mgrit_vs_sequential": seq / w64, "mixed_vs_fp64": w64 / w32}), flush=True)


# The kernel of each phase at the headline workload (names as rocprofv3 prints them).
PHASE_KERNELS = {
    "fine_relax": "wstep_kernel<32, 1, 3, 2, 512, double>",
    "coarse": "wstep_kernel<32, 2, 3, 3, 512, double>",
    "final": "wstep_kernel<32, 1, 3, 2, 512, double>",
}
PHASE_TEXT = {
    "fine_relax": "level-0 F/C relaxation and C-point residual: SDIRK3 steps, R as a polynomial in the stage "
                  "solve, each periodic banded solve by truncated-carry recurrences (windowed step kernel)",
    "coarse": "coarse levels, one launch per pass: corrected semi-Lagrangian step + periodic banded solve by "
              "truncated-carry recurrences (windowed step kernel)",
    "final": "final F-relaxation writing the space-time solution (windowed step kernel)",
}


def solve_bench(wl, steps, warmup, profile_dominant=True):
    """Time `steps` complete solves of workload wl after `warmup` untimed ones;
    per-phase GPU time from a few untimed solves with every phase bracketed
    by events, then the dominant phase's launches timed live (with the
    library's event profiler, on its stream) during the timed solves."""
    import torch
    from paper_2209_06916_amd import inputs, mgrit
    dev = torch.device("cuda:0")
    nx, nt = wl["nx"], wl["nt"]
    u0 = inputs.u0_fourier(nx, wl["seed"])
    u0_d = torch.from_numpy(u0).to(dev)
    v0_d = torch.from_numpy(inputs.initial_iterate(nt, nx, u0, wl["seed"])).to(dev)
    out = torch.empty((nt + 1, nx), dtype=torch.float64, device=dev)
    prob = mgrit.make_problem(nx, nt, wl["cfl"], wl["p"], wl["kind"], wl["q"])
    opts = mgrit.make_options(wl["ms"], max_levels=len(wl["ms"]) + 1, rtol=1e-10, max_iter=30)
    solver = mgrit.Solver(prob, opts)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        solver.solve(u0_d, v0_d, u_out=out)
    torch.cuda.synchronize()

    solver.profile_enable(["fine_relax", "coarse", "final"])
    solver.profile_read(reset=True)
    nphase = max(3, min(warmup, 5))
    for _ in range(nphase):
        solver.solve(u0_d, v0_d, u_out=out)
    torch.cuda.synchronize()
    phase_prof = solver.profile_read(reset=True)
    dom = max(phase_prof, key=lambda k: phase_prof[k]["total_ms"])
    solver.profile_enable([dom] if profile_dominant else [])
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    iters = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        starts[k].record(stream)
        info = solver.solve(u0_d, v0_d, u_out=out)
        ends[k].record(stream)
        iters.append(info["iterations"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = solver.profile_read(reset=True)
    solver.profile_enable([])
    lat_ms = np.array([a.elapsed_time(b) for a, b in zip(starts, ends)])

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
    err = (torch.linalg.vector_norm(out - seq_out) / torch.linalg.vector_norm(seq_out)).item()
    del seq_out

    # the final-time-only variant: the same solve without the final F-pass
    # (u(t_nt) is a C-point), for callers that need only the last state
    fin = torch.empty((nx,), dtype=torch.float64, device=dev)
    nfin = max(3, steps // 5)
    solver.solve(u0_d, v0_d, u_final=fin)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(nfin):
        solver.solve(u0_d, v0_d, u_final=fin)
    torch.cuda.synchronize()
    fin_s = (time.perf_counter() - t2) / nfin
    solver.close()
    del out, v0_d
    torch.cuda.empty_cache()

    dof = nx * nt
    it = int(np.median(iters))
    res = dict(wall=wall, steps=steps, iterations=it, lat_ms=lat_ms, seq_s=seq_s, fin_s=fin_s, dof=dof,
               err_vs_sequential=err, phase_ms={k: v["total_ms"] / nphase for k, v in phase_prof.items()
                                                 if v["launches"]})
    if profile_dominant:
        # Work per solve over kernel time per solve.  The coarse phase also
        # counts the launches of the last iteration's correction, queued before
        # the stopping test is known and returning at once: they add time, no work.
        flops_s, bytes_s, _ = phase_work(wl, it)[dom]
        launches = prof[dom]["launches"] / steps
        avg_s = prof[dom]["total_ms"] / prof[dom]["launches"] / 1e3
        res.update(dom=dom, launches=launches, avg_s=avg_s, flops=flops_s / launches, bytes=bytes_s / launches)
    return res


def roofline(wl, r):
    flops, bytes_, avg_s, dom = r["flops"], r["bytes"], r["avg_s"], r["dom"]
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
        if t.get("source_hash") == kernel_source_hash() and t.get("workload") == wl["name"]:
            traffic = t.get("phases", {}).get(dom, {}).get("bytes_per_launch")
    roof["traffic"] = traffic
    roof["kernel"] = PHASE_KERNELS[dom] + ": " + PHASE_TEXT[dom]
    roof["phase"] = dom
    roof["avg_launch_us"] = avg_s * 1e6
    roof["launches_per_solve"] = r["launches"]
    roof["algorithmic_flops_per_launch"] = flops
    roof["algorithmic_bytes_per_launch"] = bytes_
    return roof


def mixed_bench(wl, steps):
    """The headline workload in mixed precision: float32 inner MGRIT cycles on
    the correction equation inside float64 refinement (full space-time
    residual, update and stopping test on the GPU), to 1e-12 of the first
    full space-time residual (it carries the random F-points, so this gives
    the float64 solve's solution error); error against float64 sequential
    stepping on the GPU."""
    import torch
    from paper_2209_06916_amd import inputs, mgrit
    dev = torch.device("cuda:0")
    nx, nt = wl["nx"], wl["nt"]
    u0 = inputs.u0_fourier(nx, wl["seed"])
    u0_d = torch.from_numpy(u0).to(dev)
    v0_d = torch.from_numpy(inputs.initial_iterate(nt, nx, u0, wl["seed"])).to(dev)
    prob = mgrit.make_problem(nx, nt, wl["cfl"], wl["p"], wl["kind"], wl["q"])
    s = mgrit.Solver(prob, mgrit.make_options(wl["ms"], max_levels=len(wl["ms"]) + 1, rtol=1e-12, max_iter=30,
                                              precision="mixed"))
    out = torch.empty((nt + 1, nx), dtype=torch.float64, device=dev)
    info = s.solve(u0_d, v0_d, u_out=out)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        info = s.solve(u0_d, v0_d, u_out=out)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t) / steps
    ref = torch.empty_like(out)
    s.sequential(u0_d, ref)
    err = (torch.linalg.vector_norm(out - ref) / torch.linalg.vector_norm(ref)).item()
    s.close()
    del out, ref, v0_d
    torch.cuda.empty_cache()
    return {"ms_per_solve": 1e3 * wall, "dof_per_s": nx * nt / wall, "status": info["status"],
            "outer_iterations": info["iterations"], "inner_iterations": info["inner_iterations"],
            "rel_l2_error_vs_sequential": err}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline workload (no mixed-precision and 4096 x 4096 keys); with --serve: "
                         "no mixed-precision stream")
    ap.add_argument("--probe-workload", choices=sorted(WORKLOADS), default="config3",
                    help="the workload the --traffic-probe solves run (default: the headline)")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="for hardware-counter runs: a few solves plus one elementwise copy of "
                         "COPY_BYTES read + COPY_BYTES written (the counter calibration)")
    ap.add_argument("--serve", type=int, metavar="N", default=0,
                    help="the request-loop benchmark (N independent solves) instead of the single-solve one")
    ap.add_argument("--twod", action="store_true",
                    help="the 2D extension (config 4) against 2D sequential stepping instead of the single-solve bench")
    ap.add_argument("--precision", action="store_true",
                    help="float64 against mixed-precision MGRIT on configs 2 and 3 instead of the single-solve bench")
    ap.add_argument("--gmres", action="store_true",
                    help="exact against GMRES coarse solves (Sec. 6.3) on the Table 3 grid and configs 2 and 3")
    ap.add_argument("--summarize-profiles", metavar="DIR",
                    help="CPU only: turn the rocprofv3 runs under DIR into the profiles/ summaries")
    args = ap.parse_args()
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (the path is a single-GPU build); "
                                   f"--gpus {args.gpus} is not supported"}))
        sys.exit(2)

    import torch
    if args.serve:
        serve_bench(args.serve, seed=1005, with_mixed=not args.no_extras)
        return
    if args.precision:
        precision_bench(max(1, min(args.steps, 5)))
        return
    if args.twod:
        twod_bench(max(1, min(args.steps, 5)))
        return
    if args.gmres:
        gmres_bench(max(1, min(args.steps, 3)))
        return

    wl = HEADLINE
    if args.traffic_probe:
        wl = WORKLOADS[args.probe_workload]
        from paper_2209_06916_amd import inputs, mgrit
        dev = torch.device("cuda:0")
        u0 = inputs.u0_fourier(wl["nx"], wl["seed"])
        u0_d = torch.from_numpy(u0).to(dev)
        v0_d = torch.from_numpy(inputs.initial_iterate(wl["nt"], wl["nx"], u0, wl["seed"])).to(dev)
        out = torch.empty((wl["nt"] + 1, wl["nx"]), dtype=torch.float64, device=dev)
        s = mgrit.Solver(mgrit.make_problem(wl["nx"], wl["nt"], wl["cfl"], wl["p"], wl["kind"], wl["q"]),
                         mgrit.make_options(wl["ms"], max_levels=len(wl["ms"]) + 1))
        for _ in range(args.warmup + args.steps):
            s.solve(u0_d, v0_d, u_out=out)
        x = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"traffic_probe": True, "copy_bytes": COPY_BYTES, "solves": args.warmup + args.steps}),
              flush=True)
        return

    r = solve_bench(wl, args.steps, args.warmup)
    dof = r["dof"]
    value = dof * args.steps / r["wall"]
    line = {
        "metric": "space-time DOF/s to 1e-10 residual vs seq. stepping; p50/p99 solve latency",
        "value": value,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r["wall"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl["name"], "nx": wl["nx"], "nt": wl["nt"], "cfl": wl["cfl"], "scheme": wl["scheme"],
                   "hierarchy": [wl["nt"] // int(np.prod(wl["ms"][:i])) for i in range(len(wl["ms"]) + 1)],
                   "relaxation": "FCF", "coarse_operator": "semi-Lagrangian + implicit truncation correction",
                   "rtol": 1e-10},
        "iterations": r["iterations"],
        "latency_ms_p50": float(np.percentile(r["lat_ms"], 50)),
        "latency_ms_p99": float(np.percentile(r["lat_ms"], 99)),
        "sequential_gpu_dof_per_s": dof / r["seq_s"],
        "sequential_gpu_ms": r["seq_s"] * 1e3,
        "speedup_vs_sequential": value / (dof / r["seq_s"]),
        "rel_l2_error_vs_sequential": r["err_vs_sequential"],
        "final_time_only_ms": r["fin_s"] * 1e3,
        "final_time_only_dof_per_s": dof / r["fin_s"],
        "phase_ms_per_solve": r["phase_ms"],
        "roofline": roofline(wl, r),
    }
    if not args.no_extras:
        line["mixed"] = mixed_bench(wl, max(2, min(args.steps, 5)))
        line["mixed"]["speedup_vs_fp64"] = line["ms_per_step"] / line["mixed"]["ms_per_solve"]
        wl2 = WORKLOADS["config2"]
        r2 = solve_bench(wl2, max(args.steps, 20), args.warmup, profile_dominant=False)
        v2 = r2["dof"] * r2["steps"] / r2["wall"]
        line["config2"] = {"workload": wl2["name"], "dof_per_s": v2, "ms_per_solve": 1e3 * r2["wall"] / r2["steps"],
                           "iterations": r2["iterations"], "sequential_gpu_ms": r2["seq_s"] * 1e3,
                           "speedup_vs_sequential": v2 / (r2["dof"] / r2["seq_s"]),
                           "latency_ms_p50": float(np.percentile(r2["lat_ms"], 50)),
                           "latency_ms_p99": float(np.percentile(r2["lat_ms"], 99)),
                           "phase_ms_per_solve": r2["phase_ms"]}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
