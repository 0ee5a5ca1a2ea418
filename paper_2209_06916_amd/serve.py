"""Request loop that keeps many independent advection solves in flight on one GPU.

Each request is one MGRIT solve (its own problem, options and initial data,
zero initial iterate).  Requests are admitted in arrival order while the
device memory of the in-flight ones (the handle's workspace, u0 and the
final-time row) stays within a budget.  Every admitted request gets its own
handle and HIP stream and is advanced one MGRIT iteration at a time
(mgrit_solve_advance never blocks), so the kernels of all in-flight solves
overlap on the GPU and a request that finishes makes room for the next one
at once (continuous batching).  The coarse levels of a single solve occupy
only a few compute units, which is what concurrency recovers.

A handle's device workspace is a tensor from PyTorch's caching allocator,
handed to mgrit_setup_ws, so admitting and retiring requests never calls
hipMalloc or hipFree (hipFree would wait for every solve in flight).  Every
step of every solve runs in the HIP library; this module only schedules.
"""
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np
import torch

from . import mgrit


@dataclass
class Request:
    """One solve: u_t + u_x = 0 on [-1, 1) with the given mesh, scheme and MGRIT options."""
    nx: int
    nt: int
    p: int
    c: float
    m: int
    u0: np.ndarray
    kind: str = "erk"
    q: int = None
    min_coarse_nt: int = 8
    max_levels: int = 16
    arrival: float = 0.0  # seconds after the start of the run
    tag: object = None
    precision: str = "fp64"  # "mixed": float32 inner cycles in float64 refinement
    rtol: float = None  # default: 1e-10 of the float64 C-point residual; 1e-12 of the mixed-precision
    #                     full space-time residual, which gives the same solution error

    def problem(self):
        return mgrit.make_problem(self.nx, self.nt, self.c, self.p, self.kind, self.q)

    def options(self):
        return mgrit.make_options([self.m], max_levels=self.max_levels, min_coarse_nt=self.min_coarse_nt,
                                  coarse_launch=1, tile_tune=1, precision=self.precision,
                                  rtol=self.rtol if self.rtol is not None else (1e-12 if self.precision == "mixed"
                                                                                else 1e-10))


@dataclass
class Result:
    tag: object
    status: int
    iterations: int
    u_final: np.ndarray
    t_arrival: float
    t_admit: float
    t_done: float
    dof: int = 0
    res_history: list = field(default_factory=list)

    @property
    def latency(self):
        return self.t_done - self.t_arrival


class Server:
    """Continuous-batching request loop.

    budget_bytes bounds the device memory of the requests in flight;
    max_inflight bounds their number (one HIP stream each); setup_threads
    host threads run mgrit_setup_ws (ctypes releases the interpreter lock
    for the call, so setups overlap each other and the launch loop)."""

    def __init__(self, budget_bytes=64 << 30, max_inflight=16, device="cuda:0", setup_threads=8):
        self.budget = int(budget_bytes)
        self.max_inflight = int(max_inflight)
        self.setup_threads = int(setup_threads)
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(self.max_inflight)]

    @staticmethod
    def workspace(req):
        return mgrit.workspace_bytes(req.problem(), req.options())

    @staticmethod
    def footprint(req):
        return Server.workspace(req) + 2 * req.nx * 8

    def _setup(self, req, stream, ws):
        with torch.cuda.device(self.device):
            return mgrit.Solver(req.problem(), req.options(), stream=stream, workspace=ws)

    def run(self, requests, realtime=True):
        """Serve `requests` (arrival times honoured when realtime); returns one
        Result per request, in completion order.  A request that fails (at
        setup or in the solve) gets a Result with its status and no u_final;
        the others are not affected."""
        pending = sorted(requests, key=lambda r: r.arrival)
        for r in pending:
            if self.footprint(r) > self.budget:
                raise ValueError(f"request {r.tag} needs more than the whole budget")
        preparing, active, results = [], [], []
        free_streams = list(self.streams)
        used = 0
        t0 = time.perf_counter()

        def retire(a, status, iterations=0, hist=(), u_final=None):
            nonlocal used
            req = a["req"]
            results.append(Result(tag=req.tag, status=status, iterations=iterations, u_final=u_final,
                                  t_arrival=req.arrival, t_admit=a["t_admit"], t_done=time.perf_counter() - t0,
                                  dof=req.nx * req.nt, res_history=list(hist)))
            if a.get("solver") is not None:
                a["solver"].close()  # the stream is idle: the workspace returns to the caching allocator
            used -= a["need"]
            free_streams.append(a["stream"])

        with ThreadPoolExecutor(max_workers=self.setup_threads) as pool:
            while pending or preparing or active:
                now = time.perf_counter() - t0
                progressed = False
                # admit in arrival order while memory and slots allow; the
                # host-side setup runs on the pool
                while pending and len(active) + len(preparing) < self.max_inflight and \
                        (not realtime or pending[0].arrival <= now):
                    req = pending[0]
                    need = self.footprint(req)
                    if used + need > self.budget:
                        break
                    pending.pop(0)
                    used += need
                    stream = free_streams.pop()
                    with torch.cuda.stream(stream):
                        host = torch.from_numpy(np.ascontiguousarray(req.u0, dtype=np.float64)).pin_memory()
                        u0 = host.to(self.device, non_blocking=True)
                        ufin = torch.empty(req.nx, dtype=torch.float64, device=self.device)
                        ws = torch.empty(self.workspace(req), dtype=torch.uint8, device=self.device)
                    fut = pool.submit(self._setup, req, stream, ws)
                    preparing.append(dict(req=req, fut=fut, stream=stream, u0=u0, ufin=ufin, need=need,
                                          t_admit=time.perf_counter() - t0))
                    progressed = True
                # start the solves whose setup has finished
                for a in [a for a in preparing if a["fut"].done()]:
                    preparing.remove(a)
                    progressed = True
                    try:
                        a["solver"] = a["fut"].result()
                        a["solver"].solve_start(a["u0"], None, None, a["ufin"])
                    except mgrit.MgritError as e:
                        a["stream"].synchronize()
                        retire(a, e.status)
                        continue
                    active.append(a)
                # advance every in-flight solve by at most one iteration
                for a in list(active):
                    try:
                        done = a["solver"].solve_advance()
                        if done:
                            info = a["solver"].solve_finish(allow=_ANY_STATUS)
                    except mgrit.MgritError as e:
                        done, info = True, dict(status=e.status, iterations=0, res_history=[])
                    if not done:
                        continue
                    a["stream"].synchronize()
                    ok = info["status"] in (mgrit.OK, mgrit.ENOTCONVERGED)
                    active.remove(a)
                    retire(a, info["status"], info["iterations"], info["res_history"],
                           a["ufin"].cpu().numpy() if ok else None)
                    progressed = True
                if not progressed:
                    if realtime and not active and not preparing and pending:
                        time.sleep(min(1e-3, max(0.0, pending[0].arrival - (time.perf_counter() - t0))))
                    else:
                        time.sleep(0)  # let the setup threads take the interpreter
        return results


_ANY_STATUS = (mgrit.OK, mgrit.ENOTCONVERGED, mgrit.EINVAL, mgrit.EUNSTABLE, mgrit.ENOMEM, mgrit.EDEVICE,
               mgrit.EDIVERGED)


def synthetic_stream(n, seed, rate_hz, sizes=(256, 512, 1024, 2048, 4096, 8192), orders=(1, 3, 5), ms=(4, 8, 16),
                     cfl=(0.5, 0.9), precision="fp64"):
    """Seeded request mix: nx, nt drawn from `sizes`, upwind order p from
    `orders` with ERKp, CFL uniform in `cfl`, coarsening factor from `ms`,
    u0 a seeded 16-mode Fourier sum, Poisson arrivals at `rate_hz`."""
    from . import inputs
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for i in range(n):
        nx = int(rng.choice(sizes))
        nt = int(rng.choice(sizes))
        p = int(rng.choice(orders))
        c = float(rng.uniform(*cfl))
        m = int(rng.choice(ms))
        while nt % m:
            m //= 2
        t += rng.exponential(1.0 / rate_hz) if rate_hz > 0 else 0.0
        reqs.append(Request(nx=nx, nt=nt, p=p, c=c, m=m, u0=inputs.u0_fourier(nx, seed * 100003 + i), arrival=t,
                            tag=i, precision=precision))
    return reqs


class ThreadedServer(Server):
    """The same admission rules, with one host thread per request in flight:
    each thread sets up its handle, runs the whole solve with one blocking
    mgrit_solve call on its own stream (ctypes drops the interpreter lock
    for the call) and retires it.  Launch work is spread over the threads
    instead of one polling loop."""

    def run(self, requests, realtime=True):
        import threading
        pending = sorted(requests, key=lambda r: r.arrival)
        for r in pending:
            if self.footprint(r) > self.budget:
                raise ValueError(f"request {r.tag} needs more than the whole budget")
        cv = threading.Condition()
        state = dict(used=0, active=0)
        free_streams = list(self.streams)
        results = []
        t0 = time.perf_counter()

        def work(req, need, stream, t_admit):
            status, iters, hist, u_final = mgrit.EDEVICE, 0, [], None
            try:
                with torch.cuda.device(self.device), torch.cuda.stream(stream):
                    host = torch.from_numpy(np.ascontiguousarray(req.u0, dtype=np.float64)).pin_memory()
                    u0 = host.to(self.device, non_blocking=True)
                    ufin = torch.empty(req.nx, dtype=torch.float64, device=self.device)
                    ws = torch.empty(self.workspace(req), dtype=torch.uint8, device=self.device)
                    solver = None
                    try:
                        solver = mgrit.Solver(req.problem(), req.options(), stream=stream, workspace=ws)
                        info = solver.solve(u0, u_final=ufin, allow=_ANY_STATUS)
                        status, iters, hist = info["status"], info["iterations"], info["res_history"]
                        if status in (mgrit.OK, mgrit.ENOTCONVERGED):
                            u_final = ufin.cpu().numpy()
                    except mgrit.MgritError as e:
                        status = e.status
                    finally:
                        stream.synchronize()
                        if solver is not None:
                            solver.close()
            finally:
                with cv:
                    results.append(Result(tag=req.tag, status=status, iterations=iters, u_final=u_final,
                                          t_arrival=req.arrival, t_admit=t_admit, t_done=time.perf_counter() - t0,
                                          dof=req.nx * req.nt, res_history=list(hist)))
                    state["used"] -= need
                    state["active"] -= 1
                    free_streams.append(stream)
                    cv.notify_all()

        threads = []
        with cv:
            while pending:
                req = pending[0]
                need = self.footprint(req)
                now = time.perf_counter() - t0
                if realtime and req.arrival > now:
                    cv.wait(timeout=req.arrival - now)
                    continue
                if state["active"] >= self.max_inflight or state["used"] + need > self.budget:
                    cv.wait()
                    continue
                pending.pop(0)
                state["used"] += need
                state["active"] += 1
                stream = free_streams.pop()
                th = threading.Thread(target=work, args=(req, need, stream, time.perf_counter() - t0), daemon=True)
                th.start()
                threads.append(th)
        for th in threads:
            th.join()
        return results
