"""GPU: the request loop (paper_2209_06916_amd.serve) keeps several solves in
flight, each on its own stream through mgrit_solve_start / _advance / _finish.
Every result must be the same alone and in the mix (same bits: the solves
share no data and the kernels are deterministic), and match the oracle."""
import numpy as np
import pytest
import torch

from oracle import discretization as disc
from oracle import mgrit as omg
from paper_2209_06916_amd import inputs, mgrit, serve

pytestmark = pytest.mark.gpu


def _announce(*args):
    print("CASE", *args, flush=True)


def _mix():
    reqs = serve.synthetic_stream(7, seed=5, rate_hz=0, sizes=(256, 512, 1024), orders=(1, 3, 5), ms=(4, 8))
    reqs.append(serve.Request(nx=4096, nt=512, p=3, c=0.85, m=8, u0=inputs.u0_fourier(4096, 77), tag="big"))
    return reqs


def _by_tag(results):
    return {r.tag: r for r in results}


def test_results_are_the_same_alone_and_in_the_mix():
    _announce("serving alone vs mix")
    reqs = _mix()
    alone = _by_tag(serve.Server(max_inflight=1).run(reqs, realtime=False))
    mixed = _by_tag(serve.Server(max_inflight=len(reqs)).run(reqs, realtime=False))
    assert set(alone) == set(mixed) == {r.tag for r in reqs}
    for tag in alone:
        a, b = alone[tag], mixed[tag]
        assert a.status == b.status == mgrit.OK, tag
        assert a.iterations == b.iterations, tag
        assert a.res_history == b.res_history, tag
        np.testing.assert_array_equal(a.u_final, b.u_final)


def test_served_results_match_the_oracle():
    _announce("serving vs oracle")
    reqs = _mix()[:4]
    got = _by_tag(serve.Server(max_inflight=4).run(reqs, realtime=False))
    for r in reqs:
        ms = omg.coarsening_schedule(r.nt, r.m, r.min_coarse_nt)
        H = omg.Hierarchy(r.nx, r.nt, r.p, "erk", r.p, r.c, ms)
        v0 = np.zeros((r.nt + 1, r.nx))
        v0[0] = r.u0
        ref, info = omg.solve(H, r.u0, v0, rtol=1e-10, max_iter=30)
        g = got[r.tag]
        assert g.iterations == info["iterations"], r.tag
        assert np.linalg.norm(g.u_final - ref[-1]) <= 1e-12 * np.linalg.norm(ref[-1]), r.tag


def test_memory_budget_serialises_admission():
    """A budget that holds one request at a time still serves every request,
    with the same results."""
    _announce("serving budget")
    reqs = _mix()[:5]
    one = max(serve.Server.footprint(r) for r in reqs)
    tight = _by_tag(serve.Server(budget_bytes=one, max_inflight=8).run(reqs, realtime=False))
    free = _by_tag(serve.Server(max_inflight=8).run(reqs, realtime=False))
    for tag in free:
        np.testing.assert_array_equal(tight[tag].u_final, free[tag].u_final)
    # the requests in flight at any admission never exceeded the budget
    fp = {r.tag: serve.Server.footprint(r) for r in reqs}
    for t in tight:
        t0 = tight[t].t_admit
        live = sum(fp[u] for u in tight if tight[u].t_admit <= t0 < tight[u].t_done)
        assert live <= one
