"""GPU: mgrit_solve_noalloc (the allocation-free float64 solve, through the C
ABI) against mgrit_setup + mgrit_solve on the same seeded inputs: identical
iteration counts and residual histories, and the same solution (the same
kernels run, so the bar of the parity tests, <= 1e-12 per time point, holds
with room to spare).  Two calls in a row, the second smaller, so the second
runs in the static workspace the first left behind; then the size limit."""
import numpy as np
import pytest
import torch

from paper_2209_06916_amd import inputs, mgrit

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def _case(nx, nt, p, kind, q, c, ms, seed):
    print("CASE noalloc", nx, nt, p, kind, q, c, ms, flush=True)
    u0 = inputs.u0_fourier(nx, seed)
    v0 = inputs.initial_iterate(nt, nx, u0, seed)
    prob = mgrit.make_problem(nx, nt, c, p, kind, q)
    opts = mgrit.make_options(ms, max_levels=len(ms) + 1)
    out_a = torch.empty((nt + 1, nx), dtype=torch.float64, device=DEV)
    fin_a = torch.empty((nx,), dtype=torch.float64, device=DEV)
    info_a = mgrit.solve_noalloc(prob, opts, _t(u0), _t(v0), u_out=out_a, u_final=fin_a)
    torch.cuda.synchronize()
    s = mgrit.Solver(prob, opts)
    out_b = torch.empty_like(out_a)
    info_b = s.solve(_t(u0), _t(v0), u_out=out_b)
    torch.cuda.synchronize()
    s.close()
    a, b = out_a.cpu().numpy(), out_b.cpu().numpy()
    assert info_a["status"] == info_b["status"] == mgrit.OK
    assert info_a["iterations"] == info_b["iterations"]
    np.testing.assert_allclose(info_a["res_history"], info_b["res_history"], rtol=1e-13)
    per_t = np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)
    assert np.max(per_t) <= 1e-12, np.max(per_t)
    np.testing.assert_array_equal(fin_a.cpu().numpy(), a[-1])


def test_noalloc_matches_mgrit_solve_twice_then_smaller():
    _case(2048, 1024, 3, "erk", 3, 0.85, [8, 8, 8], 1301)
    _case(256, 256, 3, "sdirk", 3, 2.0, [4, 4], 1302)


def test_noalloc_rejects_problems_beyond_its_workspace():
    print("CASE noalloc limit", flush=True)
    nx, nt = 16384, 4096
    prob = mgrit.make_problem(nx, nt, 0.5, 5, "sdirk", 3)
    opts = mgrit.make_options([16, 16], max_levels=3)
    assert mgrit.workspace_bytes(prob, opts) > 64 << 20
    u0 = torch.zeros(nx, dtype=torch.float64, device=DEV)
    with pytest.raises(mgrit.MgritError) as ei:
        mgrit.solve_noalloc(prob, opts, u0)
    assert ei.value.status == mgrit.EINVAL
    assert "allocation-free" in str(ei.value)
    with pytest.raises(mgrit.MgritError) as ei:
        mgrit.solve_noalloc(mgrit.make_problem(256, 64, 0.85, 3), mgrit.make_options(4, precision="mixed"),
                            torch.zeros(256, dtype=torch.float64, device=DEV))
    assert ei.value.status == mgrit.EINVAL
