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


def test_caller_workspace_gives_the_same_solve():
    """mgrit_setup_ws carves the handle's buffers from a caller tensor; the
    solve is bitwise the one of a handle that allocates its own."""
    _announce("setup_ws vs setup")
    for nx, nt, p, m in [(1024, 512, 3, 8), (512, 768, 5, 4), (4096, 256, 1, 16)]:
        pr = mgrit.make_problem(nx, nt, 0.8, p, "erk")
        op = mgrit.make_options([m], max_levels=16, min_coarse_nt=8)
        u0 = torch.from_numpy(inputs.u0_fourier(nx, nx + nt)).cuda()
        outs = []
        for use_ws in (False, True):
            ws = torch.empty(mgrit.workspace_bytes(pr, op), dtype=torch.uint8, device="cuda") if use_ws else None
            s = mgrit.Solver(pr, op, workspace=ws)
            uf = torch.empty(nx, dtype=torch.float64, device="cuda")
            info = s.solve(u0, u_final=uf)
            torch.cuda.synchronize()
            outs.append((info["iterations"], uf.cpu().numpy()))
            s.close()
        assert outs[0][0] == outs[1][0]
        np.testing.assert_array_equal(outs[0][1], outs[1][1])


def test_caller_workspace_is_checked():
    _announce("setup_ws checks")
    pr = mgrit.make_problem(1024, 512, 0.8, 3, "erk")
    op = mgrit.make_options([8], max_levels=16, min_coarse_nt=8)
    need = mgrit.workspace_bytes(pr, op)
    small = torch.empty(4096, dtype=torch.uint8, device="cuda")
    with pytest.raises(mgrit.MgritError) as e:
        mgrit.Solver(pr, op, workspace=small)
    assert e.value.status == mgrit.EINVAL
    big = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(mgrit.MgritError) as e:
        mgrit.Solver(pr, op, workspace=big[1:])  # misaligned view
    assert e.value.status == mgrit.EINVAL


def test_a_failing_request_does_not_affect_the_others():
    """ERK1+U1 at CFL 1.2 is above its stability limit: that request ends with
    MGRIT_EUNSTABLE and no result; the rest are served as when alone."""
    _announce("serving failure isolation")
    reqs = _mix()[:4]
    bad = serve.Request(nx=512, nt=256, p=1, c=1.2, m=4, u0=inputs.u0_fourier(512, 9), tag="unstable")
    got = _by_tag(serve.Server(max_inflight=4).run(reqs + [bad], realtime=False))
    assert got["unstable"].status == mgrit.EUNSTABLE and got["unstable"].u_final is None
    alone = _by_tag(serve.Server(max_inflight=1).run(reqs, realtime=False))
    for r in reqs:
        assert got[r.tag].status == mgrit.OK
        np.testing.assert_array_equal(got[r.tag].u_final, alone[r.tag].u_final)


def test_threaded_server_gives_the_same_results_and_respects_the_budget():
    _announce("threaded server")
    reqs = _mix()
    alone = _by_tag(serve.Server(max_inflight=1).run(reqs, realtime=False))
    thr = _by_tag(serve.ThreadedServer(max_inflight=len(reqs)).run(reqs, realtime=False))
    for tag in alone:
        assert thr[tag].status == mgrit.OK and thr[tag].iterations == alone[tag].iterations
        np.testing.assert_array_equal(thr[tag].u_final, alone[tag].u_final)
    small = reqs[:5]
    one = max(serve.Server.footprint(r) for r in small)
    tight = _by_tag(serve.ThreadedServer(budget_bytes=one, max_inflight=8).run(small, realtime=False))
    fp = {r.tag: serve.Server.footprint(r) for r in small}
    for t in tight:
        t0 = tight[t].t_admit
        assert sum(fp[u] for u in tight if tight[u].t_admit <= t0 < tight[u].t_done) <= one
    bad = serve.Request(nx=512, nt=256, p=1, c=1.2, m=4, u0=inputs.u0_fourier(512, 9), tag="unstable")
    got = _by_tag(serve.ThreadedServer(max_inflight=4).run(small + [bad], realtime=False))
    assert got["unstable"].status == mgrit.EUNSTABLE and got["unstable"].u_final is None


def test_threaded_server_serves_mixed_precision_requests():
    """Mixed-precision requests (float32 inner cycles in float64 refinement)
    reach the float64 oracle's sequential solution to 1e-10."""
    _announce("serving mixed")
    reqs = serve.synthetic_stream(6, seed=8, rate_hz=0, sizes=(256, 512, 1024), orders=(1, 3, 5), ms=(4, 8),
                                  precision="mixed")
    got = _by_tag(serve.ThreadedServer(max_inflight=6).run(reqs, realtime=False))
    for r in reqs:
        assert got[r.tag].status == mgrit.OK, r.tag
        ref = omg.sequential(disc.MOLStep(r.p, "erk", r.p, r.c), r.u0, r.nt)[-1]
        assert np.linalg.norm(got[r.tag].u_final - ref) <= 1e-10 * np.linalg.norm(ref), r.tag


def test_polling_server_serves_mixed_precision_requests():
    """The single-thread polling loop drives mixed-precision handles through
    mgrit_solve_start/_advance and gives the threaded loop's bits."""
    _announce("serving mixed, polling loop")
    reqs = serve.synthetic_stream(5, seed=9, rate_hz=0, sizes=(256, 512), orders=(1, 3, 5), ms=(4, 8),
                                  precision="mixed")
    polled = _by_tag(serve.Server(max_inflight=5).run(reqs, realtime=False))
    threaded = _by_tag(serve.ThreadedServer(max_inflight=5).run(reqs, realtime=False))
    for r in reqs:
        assert polled[r.tag].status == mgrit.OK, r.tag
        np.testing.assert_array_equal(polled[r.tag].u_final, threaded[r.tag].u_final)
        ref = omg.sequential(disc.MOLStep(r.p, "erk", r.p, r.c), r.u0, r.nt)[-1]
        assert np.linalg.norm(polled[r.tag].u_final - ref) <= 1e-10 * np.linalg.norm(ref), r.tag
