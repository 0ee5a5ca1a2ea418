"""GPU parity: every entry point of libmgrit (called through the C ABI) against
the FP64 CPU oracle on the same seeded inputs.

Tolerances: single operator applications and sequential stepping are compared
elementwise at 1e-13 relative to the vector's max-norm (different but exact
algorithms: banded recurrences on the GPU, FFT diagonalisation in the oracle;
Horner forms on the GPU, Butcher stages in the oracle).  Full MGRIT solves: the
identical iteration count, relative L2 error per C-point <= 1e-12, and the
residual history within 1e-8 relative (the last entries are ~1e-10 of the
first, so their absolute agreement is much tighter).
"""
import numpy as np
import pytest
import torch

from oracle import discretization as disc
from oracle import mgrit as omg
from golden_check import check_against_golden, golden
from paper_2209_06916_amd import inputs, mgrit

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _announce(*args):
    print("CASE", *args, flush=True)


# --------------------------------------------------------------------------
# single time-stepper applications (fine Phi and coarse Psi_l)
# --------------------------------------------------------------------------

FINE_CASES = [
    (64, 1, "erk", 1, 0.85), (256, 3, "erk", 3, 1.3), (4096, 3, "erk", 3, 0.85), (1000, 5, "erk", 5, 0.9),
    (77, 3, "erk", 3, 1.0), (512, 2, "erk", 2, 0.45), (8192, 4, "erk", 4, 0.9),
    (256, 1, "sdirk", 1, 3.0), (1024, 3, "sdirk", 3, 5.0), (16384, 5, "sdirk", 3, 0.5), (1000, 5, "sdirk", 3, 0.5),
    (300, 2, "sdirk", 2, 2.0), (5, 1, "erk", 1, 0.5), (3, 3, "sdirk", 3, 1.5),
]


@pytest.mark.parametrize("nx,p,kind,q,c", FINE_CASES)
def test_fine_step_matches_oracle(nx, p, kind, q, c):
    _announce("fine", nx, p, kind, q, c)
    rng = np.random.default_rng(nx + p)
    count, nsteps = 3, 4
    v = rng.standard_normal((count, nx))
    s = mgrit.Solver(mgrit.make_problem(nx, 8, c, p, kind, q), mgrit.make_options(2, coarse="ideal"))
    out = torch.empty((count, nx), dtype=torch.float64, device=DEV)
    s.apply_step(0, _t(v), out, nsteps)
    step = disc.MOLStep(p, kind, q, c)
    ref = v.copy()
    for _ in range(nsteps):
        ref = step(ref)
    got = _np(out)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) <= 1e-13 * scale * max(1.0, c)


COARSE_CASES = [
    (256, 1, "erk", 1, 0.85, [4]), (4096, 3, "erk", 3, 0.85, [8, 8, 8]), (1000, 3, "erk", 3, 1.38, [4, 4]),
    (512, 5, "erk", 5, 0.9, [16, 4, 4]), (1024, 3, "sdirk", 3, 5.0, [2, 2, 2, 2]),
    (16384, 5, "sdirk", 3, 0.5, [16, 16, 4]), (300, 5, "sdirk", 3, 0.5, [4, 4]), (64, 1, "sdirk", 1, 1.0, [16]),
]


@pytest.mark.parametrize("nx,p,kind,q,c,ms", COARSE_CASES)
def test_coarse_steps_match_oracle(nx, p, kind, q, c, ms):
    _announce("coarse", nx, p, kind, q, c, ms)
    nt = int(np.prod(ms)) * 2
    opts = mgrit.make_options(ms, max_levels=len(ms) + 1)
    s = mgrit.Solver(mgrit.make_problem(nx, nt, c, p, kind, q), opts)
    assert s.num_levels == len(ms) + 1
    recs = disc.correction_coefficients(p, kind, q, c, ms)
    rng = np.random.default_rng(7)
    v = rng.standard_normal((2, nx))
    for lev, rec in enumerate(recs, start=1):
        info = s.level_info(lev)
        assert info["K"] == rec["K"] and info["eps"] == pytest.approx(rec["eps"], abs=1e-12)
        assert info["phi_p"] == pytest.approx(rec["phi_p"], rel=1e-12, abs=1e-14)
        assert info["phi_q"] == pytest.approx(rec["phi_q"], rel=1e-12, abs=1e-14)
        out = torch.empty((2, nx), dtype=torch.float64, device=DEV)
        s.apply_step(lev, _t(v), out, 3)
        psi = disc.CorrectedSLStep(p, q, rec["shift"], rec["phi_p"], rec["phi_q"])
        ref = psi(psi(psi(v)))
        got = _np(out)
        assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref)) * max(1.0, abs(rec["phi_p"])), lev


# the lean coarse-step kernel: 16 points per lane with nx = 1024 NW, NW = 1,
# 2, 4, 8, and one wavefront of 8 or 4 points per lane (nx = 512, 256), for
# the three (taps, recurrence order) pairs p = 1, 3, 5
LEAN_CASES = [(nx, p) for nx in (256, 512, 1024, 2048, 4096, 8192) for p in (1, 3, 5)]


@pytest.mark.parametrize("nx,p", LEAN_CASES)
def test_lean_coarse_steps_match_oracle(monkeypatch, nx, p):
    # the 16-point shapes pinned: by default setup takes 8 points per lane up
    # to nx = 2048 and the windowed kernel from nx = 8192
    monkeypatch.setenv("MGRIT_L_COARSE", "16")
    monkeypatch.setenv("MGRIT_NO_LEAN", "0")
    _announce("lean coarse", nx, p)
    c = {1: 0.85, 3: 1.2, 5: 0.9}[p]
    ms = [8, 16]
    s = mgrit.Solver(mgrit.make_problem(nx, 2 * 128, c, p), mgrit.make_options(ms, max_levels=3))
    recs = disc.correction_coefficients(p, "erk", p, c, ms)
    v = np.random.default_rng(nx + 11 * p).standard_normal((3, nx))
    for lev, rec in enumerate(recs, start=1):
        out = torch.empty((3, nx), dtype=torch.float64, device=DEV)
        s.apply_step(lev, _t(v), out, 5)
        psi = disc.CorrectedSLStep(p, p, rec["shift"], rec["phi_p"], rec["phi_q"])
        ref = v
        for _ in range(5):
            ref = psi(ref)
        got = _np(out)
        assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref)) * max(1.0, abs(rec["phi_p"])), lev


@pytest.mark.parametrize("case", [
    dict(nx=1024, nt=256, p=1, kind="erk", q=1, c=0.85, ms=[4, 4, 4]),
    dict(nx=2048, nt=128, p=5, kind="erk", q=5, c=0.9, ms=[4, 8]),
    dict(nx=1024, nt=128, p=3, kind="sdirk", q=3, c=5.0, ms=[4, 4]),
    dict(nx=8192, nt=64, p=3, kind="erk", q=3, c=0.85, ms=[4, 4]),
    dict(nx=256, nt=512, p=3, kind="erk", q=3, c=0.7, ms=[4, 4, 4]),
    dict(nx=512, nt=256, p=5, kind="erk", q=5, c=0.9, ms=[8, 4]),
    dict(nx=512, nt=128, p=1, kind="sdirk", q=1, c=2.0, ms=[4, 4]),
])
def test_lean_full_solve_matches_oracle(case):
    _announce("lean solve", case)
    s, info, got, fin, ref, rinfo = _solve_both(case["nx"], case["nt"], case["p"], case["kind"], case["q"],
                                                case["c"], case["ms"], u0kind="fourier")
    _check_parity(info, got, fin, ref, rinfo, case["ms"][0])


@pytest.mark.parametrize("nx,p", [(1024, 3), (2048, 5), (4096, 1), (4096, 3)])
def test_lean_eight_point_shapes_match_oracle(monkeypatch, nx, p):
    """Chunks of 8 points on 2, 4 and 8 wavefronts (MGRIT_L_COARSE=8): single
    coarse steps and a full V-cycle solve against the oracle."""
    _announce("lean L=8", nx, p)
    monkeypatch.setenv("MGRIT_L_COARSE", "8")
    c = {1: 0.85, 3: 1.2, 5: 0.9}[p]
    ms = [8, 8]
    s = mgrit.Solver(mgrit.make_problem(nx, 2 * 64, c, p), mgrit.make_options(ms, max_levels=3))
    recs = disc.correction_coefficients(p, "erk", p, c, ms)
    v = np.random.default_rng(nx + 13 * p).standard_normal((3, nx))
    for lev, rec in enumerate(recs, start=1):
        out = torch.empty((3, nx), dtype=torch.float64, device=DEV)
        s.apply_step(lev, _t(v), out, 5)
        psi = disc.CorrectedSLStep(p, p, rec["shift"], rec["phi_p"], rec["phi_q"])
        ref = v
        for _ in range(5):
            ref = psi(ref)
        got = _np(out)
        assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref)) * max(1.0, abs(rec["phi_p"])), lev
    s2, info, got, fin, ref, rinfo = _solve_both(nx, 256, p, "erk", p, c, [4, 4, 4], u0kind="fourier")
    _check_parity(info, got, fin, ref, rinfo, 4)


@pytest.mark.parametrize("nx,generic_l", [(4096, "4"), (512, "2"), (256, "2")])
def test_lean_and_generic_coarse_kernels_agree(monkeypatch, nx, generic_l):
    """A chunk length outside the lean shapes selects the generic step kernel
    on the coarse levels, the default one the lean kernel; both solve the
    same system."""
    _announce("lean vs generic", nx, generic_l)
    nt = 512
    u0 = inputs.u0_fourier(nx, 31)
    v0 = _t(inputs.initial_iterate(nt, nx, u0, 31))
    outs = []
    for lc in ("16", generic_l):
        monkeypatch.setenv("MGRIT_L_COARSE", lc)
        s = mgrit.Solver(mgrit.make_problem(nx, nt, 0.85, 3), mgrit.make_options([8, 8, 8], max_levels=4))
        o = torch.empty((nt + 1, nx), dtype=torch.float64, device=DEV)
        info = s.solve(_t(u0), v0, u_out=o)
        outs.append((info["iterations"], _np(o)))
    assert outs[0][0] == outs[1][0]
    np.testing.assert_allclose(outs[0][1], outs[1][1], rtol=0, atol=1e-13 * np.max(np.abs(outs[1][1])))


@pytest.mark.parametrize("nu,ms,nx,p", [(1, [8, 8, 8], 4096, 3), (0, [4, 4], 1024, 1), (2, [4, 2, 2], 2048, 5),
                                        (1, [4, 4, 4], 512, 3), (1, [8, 4], 256, 5)])
def test_persistent_and_per_pass_coarse_cycles_agree(monkeypatch, nu, ms, nx, p):
    """The coarse part of each V-cycle as one cooperative launch with grid
    barriers and as one launch per pass: same passes, same arithmetic, so the
    same bits."""
    _announce("persistent vs per-pass", nu, ms, nx, p)
    nt = int(np.prod(ms)) * 8
    c = {1: 0.85, 3: 1.2, 5: 0.9}[p]
    u0 = inputs.u0_fourier(nx, 41)
    v0 = _t(inputs.initial_iterate(nt, nx, u0, 41))
    outs = []
    for flag in ("0", "1"):
        monkeypatch.setenv("MGRIT_NO_PERSISTENT", flag)
        s = mgrit.Solver(mgrit.make_problem(nx, nt, c, p), mgrit.make_options(ms, max_levels=len(ms) + 1, nu=nu))
        o = torch.empty((nt + 1, nx), dtype=torch.float64, device=DEV)
        info = s.solve(_t(u0), v0, u_out=o)
        outs.append((info["iterations"], info["res_history"], _np(o)))
    assert outs[0][0] == outs[1][0]
    assert outs[0][1] == outs[1][1]
    np.testing.assert_array_equal(outs[0][2], outs[1][2])


# --------------------------------------------------------------------------
# sequential stepping and the space-time residual
# --------------------------------------------------------------------------

@pytest.mark.parametrize("nx,nt,p,kind,q,c", [(256, 256, 1, "erk", 1, 0.85), (4096, 512, 3, "erk", 3, 0.85),
                                              (1000, 64, 5, "sdirk", 3, 0.5), (512, 128, 3, "sdirk", 3, 5.0),
                                              (1000, 102, 5, "erk", 5, 0.9), (77, 38, 3, "erk", 3, 1.0),
                                              (512, 130, 2, "erk", 2, 0.45), (4096, 1000, 4, "erk", 4, 0.9)])
def test_sequential_and_residual_match_oracle(nx, nt, p, kind, q, c):
    _announce("sequential", nx, nt, p, kind, q, c)
    u0 = inputs.u0_fourier(nx, seed=3)
    m = 4 if nt % 4 == 0 else 2
    s = mgrit.Solver(mgrit.make_problem(nx, nt, c, p, kind, q), mgrit.make_options(m, coarse="ideal"))
    out = torch.empty((nt + 1, nx), dtype=torch.float64, device=DEV)
    s.sequential(_t(u0), out)
    step = disc.MOLStep(p, kind, q, c)
    ref = omg.sequential(step, u0, nt)
    got = _np(out)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    # residual of a perturbed iterate
    pert = ref + 1e-3 * np.random.default_rng(1).standard_normal(ref.shape)
    r = torch.empty((nt, nx), dtype=torch.float64, device=DEV)
    n = s.residual(_t(pert), r)
    rref = omg.spacetime_residual(step, pert)
    assert np.max(np.abs(_np(r) - rref)) <= 1e-13 * np.max(np.abs(pert))
    assert n == pytest.approx(np.linalg.norm(rref), rel=1e-12)
    # the sequential solution has zero residual up to rounding
    assert s.residual(out) <= 1e-13 * np.linalg.norm(ref)


# --------------------------------------------------------------------------
# full MGRIT solves
# --------------------------------------------------------------------------

def _solve_both(nx, nt, p, kind, q, c, ms, coarse="sl_corrected", nu=1, u0kind="sin4", seed=1001,
                rtol=1e-10, max_iter=30):
    u0 = inputs.u0_sin4(nx) if u0kind == "sin4" else inputs.u0_fourier(nx, seed)
    v0 = inputs.initial_iterate(nt, nx, u0, seed)
    opts = mgrit.make_options(ms, max_levels=len(ms) + 1, nu=nu, coarse=coarse, rtol=rtol, max_iter=max_iter,
                              diverge_factor=0.0)
    s = mgrit.Solver(mgrit.make_problem(nx, nt, c, p, kind, q), opts)
    out = torch.empty((nt + 1, nx), dtype=torch.float64, device=DEV)
    fin = torch.empty((nx,), dtype=torch.float64, device=DEV)
    info = s.solve(_t(u0), _t(v0), u_out=out, u_final=fin)
    H = omg.Hierarchy(nx, nt, p, kind, q, c, ms, coarse=coarse)
    ref, rinfo = omg.solve(H, u0, v0, rtol=rtol, max_iter=max_iter, nu=nu)
    return s, info, _np(out), _np(fin), ref, rinfo


def _check_parity(info, got, fin, ref, rinfo, m):
    assert info["iterations"] == rinfo["iterations"]
    hist = np.array(info["res_history"])
    rhist = np.array(rinfo["res_history"])
    assert len(hist) == len(rhist)
    np.testing.assert_allclose(hist, rhist, rtol=1e-8, atol=1e-14 * rhist[0])
    C, Cref = got[::m], ref[::m]
    per_c = np.linalg.norm(C - Cref, axis=1) / np.linalg.norm(Cref, axis=1)
    assert np.max(per_c) <= 1e-12, np.max(per_c)
    # F-points too (the full output), same bound per time point
    per_t = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert np.max(per_t) <= 1e-12, np.max(per_t)
    np.testing.assert_array_equal(fin, got[-1])


@pytest.mark.parametrize("case", [
    # config 1: nx = nt = 256, ERK1+U1, c = 0.85, m = 4, two-level
    dict(nx=256, nt=256, p=1, kind="erk", q=1, c=0.85, ms=[4]),
    dict(nx=64, nt=256, p=3, kind="erk", q=3, c=1.38, ms=[4, 4, 4]),
    dict(nx=64, nt=256, p=3, kind="sdirk", q=3, c=5.0, ms=[8]),
    dict(nx=100, nt=128, p=5, kind="erk", q=5, c=0.9, ms=[4, 4]),
    dict(nx=96, nt=256, p=5, kind="sdirk", q=3, c=0.5, ms=[16, 4]),
    dict(nx=128, nt=64, p=1, kind="sdirk", q=1, c=1.0, ms=[2, 2, 2, 2, 2]),
    dict(nx=257, nt=96, p=3, kind="erk", q=3, c=0.85, ms=[3, 2, 2]),
])
def test_full_solve_matches_oracle(case):
    _announce("solve", case)
    s, info, got, fin, ref, rinfo = _solve_both(case["nx"], case["nt"], case["p"], case["kind"], case["q"],
                                                case["c"], case["ms"])
    _check_parity(info, got, fin, ref, rinfo, case["ms"][0])


@pytest.mark.parametrize("kind,p,c", [("erk", 1, 0.85), ("erk", 3, 0.85 * 1.62589), ("sdirk", 1, 1.0),
                                      ("sdirk", 3, 5.0)])
def test_strong_scaling_problems_match_oracle(kind, p, c):
    """The four problems of the paper's strong-scaling study (Fig. 4: ERK at
    85% of the Table 2 CFL limits, SDIRK1 at CFL 1, SDIRK3 at CFL 5; m = 16
    on the first level and 4 below, down to fewer than two coarse points
    after one more coarsening), at nx x nt = 256 x 1024 instead of
    4096 x 16384: same iterations and iterates as the oracle."""
    _announce("fig4", kind, p, c)
    s, info, got, fin, ref, rinfo = _solve_both(256, 1024, p, kind, p, c, [16, 4, 4], max_iter=60)
    assert s.num_levels == 4
    _check_parity(info, got, fin, ref, rinfo, 16)


@pytest.mark.parametrize("case", [
    dict(nx=64, nt=256, p=1, kind="sdirk", q=1, c=1.0, ms=[4], max_iter=60),
    dict(nx=96, nt=128, p=3, kind="sdirk", q=3, c=2.0, ms=[4, 4], max_iter=60),
    dict(nx=128, nt=64, p=3, kind="erk", q=3, c=0.4, ms=[2, 2], max_iter=30),
    dict(nx=64, nt=256, p=3, kind="sdirk", q=3, c=5.0, ms=[8], max_iter=6),  # diverging (LFA 2.4)
])
def test_rediscretised_coarse_operator_matches_oracle(case):
    """Coarse levels take the fine scheme at the level's step (Sec. 5): same
    iterates and residual histories as the oracle, also where the iteration
    diverges (there the last residual is ~1e3 times the first, so the
    history is compared relative to each entry)."""
    _announce("redisc", case)
    s, info, got, fin, ref, rinfo = _solve_both(case["nx"], case["nt"], case["p"], case["kind"], case["q"],
                                                case["c"], case["ms"], coarse="redisc", u0kind="fourier",
                                                max_iter=case["max_iter"])
    if case["max_iter"] == 6:
        assert info["status"] == mgrit.ENOTCONVERGED and info["iterations"] == 6 == rinfo["iterations"]
        np.testing.assert_allclose(info["res_history"], rinfo["res_history"], rtol=1e-8)
        per_c = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
        assert np.max(per_c) <= 1e-10
        return
    _check_parity(info, got, fin, ref, rinfo, case["ms"][0])


SSP43 = ([[0, 0, 0, 0], [0.5, 0, 0, 0], [0.5, 0.5, 0, 0], [1 / 6, 1 / 6, 1 / 6, 0]], [1 / 6, 1 / 6, 1 / 6, 0.5])
G23 = (3 + 3 ** 0.5) / 6
SDIRK23 = ([[G23, 0], [1 - 2 * G23, G23]], [0.5, 0.5])


@pytest.mark.parametrize("case", [
    dict(nx=256, nt=256, p=3, kind="erk", q=3, c=1.0, ms=[4, 4], tab=SSP43),
    dict(nx=2048, nt=128, p=3, kind="sdirk", q=3, c=2.0, ms=[8], tab=SDIRK23),
    dict(nx=100, nt=64, p=5, kind="erk", q=3, c=0.8, ms=[4, 4], tab=SSP43),
])
def test_caller_tableau_solves_match_oracle(case):
    """A Butcher tableau passed at the boundary (Sec. 4.2): the four-stage
    third-order SSP method and the two-stage third-order SDIRK method, fine
    steps and the correction coefficients' e_RK both from it; same
    iterations and iterates as the oracle with the same tableau."""
    c = case
    _announce("tableau", c["kind"], c["nx"], c["nt"])
    u0 = inputs.u0_fourier(c["nx"], 1401)
    v0 = inputs.initial_iterate(c["nt"], c["nx"], u0, 1401)
    s = mgrit.Solver(mgrit.make_problem(c["nx"], c["nt"], c["c"], c["p"], c["kind"], c["q"], tableau=c["tab"]),
                     mgrit.make_options(c["ms"], max_levels=len(c["ms"]) + 1))
    out = torch.empty((c["nt"] + 1, c["nx"]), dtype=torch.float64, device=DEV)
    fin = torch.empty((c["nx"],), dtype=torch.float64, device=DEV)
    info = s.solve(_t(u0), _t(v0), u_out=out, u_final=fin)
    H = omg.Hierarchy(c["nx"], c["nt"], c["p"], c["kind"], c["q"], c["c"], c["ms"], tab=c["tab"])
    ref, rinfo = omg.solve(H, u0, v0)
    _check_parity(info, _np(out), _np(fin), ref, rinfo, c["ms"][0])


def test_ideal_coarse_operator_one_iteration():
    _announce("ideal")
    s, info, got, fin, ref, rinfo = _solve_both(128, 128, 3, "erk", 3, 1.0, [8], coarse="ideal")
    assert info["iterations"] == 1 == rinfo["iterations"]
    _check_parity(info, got, fin, ref, rinfo, 8)


def test_f_relaxation_nu0_and_fcf_nu2():
    for nu in (0, 2):
        _announce("nu", nu)
        s, info, got, fin, ref, rinfo = _solve_both(64, 128, 3, "erk", 3, 1.0, [4, 4], nu=nu)
        _check_parity(info, got, fin, ref, rinfo, 4)


def test_not_converged_status_and_history():
    _announce("max_iter")
    s, info, got, fin, ref, rinfo = _solve_both(64, 128, 1, "erk", 1, 0.85, [4], max_iter=3)
    assert info["status"] == mgrit.ENOTCONVERGED
    assert info["iterations"] == 3 == rinfo["iterations"]
    _check_parity(info, got, fin, ref, rinfo, 4)


def test_uncorrected_sl_is_caught_diverging():
    """Plain SL coarse operator with ERK1+U1 at c/c_max in (1/m, 1-1/m) diverges
    (end of Sec. 5.2); the library reports it instead of looping."""
    _announce("diverge")
    nx, nt = 256, 1024
    u0 = inputs.u0_sin4(nx)
    v0 = inputs.initial_iterate(nt, nx, u0, 5)
    opts = mgrit.make_options(4, coarse="sl_plain", max_iter=200, diverge_factor=1e3)
    s = mgrit.Solver(mgrit.make_problem(nx, nt, 0.5, 1), opts)
    info = s.solve(_t(u0), _t(v0), allow=(mgrit.EDIVERGED, mgrit.ENOTCONVERGED))
    assert info["status"] in (mgrit.EDIVERGED, mgrit.ENOTCONVERGED)
    assert info["res_final"] > info["res0"] * 1e-3


def test_solve_is_deterministic():
    _announce("determinism")
    nx, nt = 512, 512
    u0 = inputs.u0_fourier(nx, 9)
    v0 = _t(inputs.initial_iterate(nt, nx, u0, 9))
    s = mgrit.Solver(mgrit.make_problem(nx, nt, 0.85, 3), mgrit.make_options(8, max_levels=4, min_coarse_nt=8))
    outs = []
    for _ in range(2):
        o = torch.empty((nt + 1, nx), dtype=torch.float64, device=DEV)
        s.solve(_t(u0), v0, u_out=o)
        outs.append(_np(o))
    np.testing.assert_array_equal(outs[0], outs[1])


def test_config2_full_size_matches_oracle():
    """nx = nt = 4096, CFL 0.85, ERK3+U3, V-cycle with m = 8 down to 8 coarse
    steps (4096 -> 512 -> 64 -> 8), seeded 16-mode Fourier u0."""
    _announce("config2 full")
    s, info, got, fin, ref, rinfo = _solve_both(4096, 4096, 3, "erk", 3, 0.85, [8, 8, 8], u0kind="fourier",
                                                seed=1002)
    _check_parity(info, got, fin, ref, rinfo, 8)


def test_config3_full_size_matches_oracle():
    """nx = nt = 16384, CFL 0.5, U5 + SDIRK3, m = 16, 16384 -> 1024 -> 64 -> 4,
    seed 1003, against the oracle's own solve of the same workload
    (tests/golden/config3_oracle.npz, written by make_config3.py)."""
    _announce("config3 full")
    g = golden("config3_oracle.npz")
    nx = nt = 16384
    u0 = inputs.u0_fourier(nx, 1003)
    v0 = inputs.initial_iterate(nt, nx, u0, 1003)
    s = mgrit.Solver(mgrit.make_problem(nx, nt, 0.5, 5, "sdirk", 3),
                     mgrit.make_options([16, 16, 16], max_levels=4))
    out = torch.empty((nt + 1, nx), dtype=torch.float64, device=DEV)
    info = s.solve(_t(u0), _t(v0), u_out=out)
    del v0
    torch.cuda.synchronize()
    assert info["status"] == mgrit.OK
    check_against_golden(info, out, g, out[::16, ::256].cpu().numpy(), 16, 77)


# --------------------------------------------------------------------------
# level-0 explicit relaxation through wavefront tiles (temporal blocking)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("tile_p", [8, 16])
@pytest.mark.parametrize("p,q,c,coarse,ms", [(1, 1, 0.85, "sl_corrected", [4]), (2, 2, 0.45, "ideal", [4]),
                                             (3, 3, 1.2, "sl_corrected", [8, 4]), (4, 4, 0.9, "ideal", [2]),
                                             (5, 5, 0.9, "sl_corrected", [4, 4])])
def test_tiled_relaxation_matches_oracle(monkeypatch, tile_p, p, q, c, coarse, ms):
    _announce("tiles", tile_p, p, q, c, coarse, ms)
    monkeypatch.setenv("MGRIT_TILE_P", str(tile_p))
    nx, nt = 300, 128
    s, info, got, fin, ref, rinfo = _solve_both(nx, nt, p, "erk", q, c, ms, coarse=coarse, u0kind="fourier")
    _check_parity(info, got, fin, ref, rinfo, ms[0])


def test_tiled_and_slab_sequential_stepping_agree(monkeypatch):
    """mgrit_sequential through blocks of tile launches and through the
    one-workgroup step kernel."""
    _announce("sequential tiles vs slab")
    nx, nt = 4096, 333
    u0 = _t(inputs.u0_fourier(nx, 23))
    outs = []
    for flag in ("0", "1"):
        monkeypatch.setenv("MGRIT_NO_TILES", flag)
        s = mgrit.Solver(mgrit.make_problem(nx, nt, 0.85, 3), mgrit.make_options(3, coarse="ideal"))
        o = torch.empty((nt + 1, nx), dtype=torch.float64, device=DEV)
        s.sequential(u0, o)
        outs.append(_np(o))
    np.testing.assert_allclose(outs[0], outs[1], rtol=0, atol=1e-13 * np.max(np.abs(outs[1])))


@pytest.mark.parametrize("written_out", ["0", "1"])
def test_tiled_and_slab_relaxation_agree(monkeypatch, written_out):
    """Level-0 relaxation through the wavefront tiles and through the
    one-workgroup step kernel.  Both apply ERK3 by Horner in Z = -c L_3 unless
    the tiles take the step written out as one 10-tap stencil, which changes
    only the rounding: then the two agree to the parity bound, 1e-12."""
    _announce("tiles vs slab", written_out)
    monkeypatch.setenv("MGRIT_TILE_COMPOSE", written_out)
    tol = 1e-14 if written_out == "0" else 1e-12
    nx, nt = 1024, 512
    u0 = inputs.u0_fourier(nx, 21)
    v0 = _t(inputs.initial_iterate(nt, nx, u0, 21))
    outs = []
    for flag in ("0", "1"):
        monkeypatch.setenv("MGRIT_NO_TILES", flag)
        s = mgrit.Solver(mgrit.make_problem(nx, nt, 0.85, 3), mgrit.make_options([8, 8], max_levels=3))
        o = torch.empty((nt + 1, nx), dtype=torch.float64, device=DEV)
        info = s.solve(_t(u0), v0, u_out=o)
        outs.append((info["iterations"], _np(o)))
    assert outs[0][0] == outs[1][0]
    np.testing.assert_allclose(outs[0][1], outs[1][1], rtol=0, atol=tol * np.max(np.abs(outs[1][1])))


@pytest.mark.parametrize("nx,nt,p,m", [(4096, 4096, 3, 8), (1024, 512, 5, 4), (2048, 256, 1, 16)])
def test_tuned_tiles_give_the_same_solve(nx, nt, p, m):
    """tile_tune = 1 times the candidate tile widths at setup and keeps the
    fastest; every width gives the same bits."""
    _announce("tile tune", nx, nt, p, m)
    u0 = _t(inputs.u0_fourier(nx, 3))
    outs = []
    for tune in (0, 1):
        s = mgrit.Solver(mgrit.make_problem(nx, nt, 0.8, p),
                         mgrit.make_options([m], max_levels=16, min_coarse_nt=8, tile_tune=tune))
        assert s.level_info(0)["tile_p"] in (8, 16)
        fin = torch.empty(nx, dtype=torch.float64, device=DEV)
        info = s.solve(u0, u_final=fin)
        outs.append((info["iterations"], _np(fin)))
    assert outs[0][0] == outs[1][0]
    np.testing.assert_array_equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("nu", [0, 2])
def test_relaxation_variants_match_oracle(nu):
    """F-relaxation (nu = 0, the paper's Fig. 6 variant) and FCFCF (nu = 2)
    against the oracle on config 1, with config 1's LFA ordering: F converges
    more slowly than FCF."""
    _announce("relaxation variant", nu)
    s, info, got, fin, ref, rinfo = _solve_both(256, 256, 1, "erk", 1, 0.85, [4], nu=nu, max_iter=60)
    _check_parity(info, got, fin, ref, rinfo, 4)
    s1, info1, *_ = _solve_both(256, 256, 1, "erk", 1, 0.85, [4], nu=1)
    if nu == 0:
        assert info["conv_factor"] > info1["conv_factor"]
        assert info["iterations"] > info1["iterations"]
    else:
        assert info["iterations"] <= info1["iterations"]


def test_persistent_cycle_on_a_large_grid_agrees(monkeypatch):
    """The persistent coarse cycle is used up to 128 workgroups by default;
    raised to 1024 it runs 512 workgroups here and gives the per-pass bits."""
    _announce("persistent large grid")
    nx, nt, ms = 256, 32768, [8, 8, 8]
    u0 = inputs.u0_fourier(nx, 43)
    v0 = _t(inputs.initial_iterate(nt, nx, u0, 43))
    outs = []
    for flag in ("0", "1"):
        monkeypatch.setenv("MGRIT_NO_PERSISTENT", flag)
        monkeypatch.setenv("MGRIT_PERSISTENT_MAX_GRID", "1024")
        s = mgrit.Solver(mgrit.make_problem(nx, nt, 0.85, 3), mgrit.make_options(ms, max_levels=4))
        fin = torch.empty(nx, dtype=torch.float64, device=DEV)
        info = s.solve(_t(u0), v0, u_final=fin)
        outs.append((info["iterations"], info["res_history"], _np(fin)))
    assert outs[0][0] == outs[1][0] and outs[0][1] == outs[1][1]
    np.testing.assert_array_equal(outs[0][2], outs[1][2])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_seeded_initial_iterate_matches_the_explicit_one(precision):
    """mgrit_solve without v_init and with options.init_seed draws the
    SplitMix64 iterate on the device: the solve equals, bit for bit, the one
    given that iterate (inputs.initial_iterate_splitmix) explicitly."""
    _announce("seed", precision)
    nx, nt, seed = 512, 256, 987654321
    u0 = inputs.u0_fourier(nx, 3)
    v0 = inputs.initial_iterate_splitmix(nt, nx, u0, seed)
    prob = mgrit.make_problem(nx, nt, 0.85, 3)
    kw = dict(max_levels=3, precision=precision, rtol=1e-10 if precision == "fp64" else 1e-12)
    outs, infos = [], []
    for v, sd in ((None, seed), (_t(v0), 0)):
        s = mgrit.Solver(prob, mgrit.make_options([4, 4], init_seed=sd, **kw))
        out = torch.empty((nt + 1, nx), dtype=torch.float64, device=DEV)
        infos.append(s.solve(_t(u0), v, u_out=out))
        outs.append(_np(out))
    assert infos[0]["iterations"] == infos[1]["iterations"]
    assert infos[0]["res_history"] == infos[1]["res_history"]
    np.testing.assert_array_equal(outs[0], outs[1])
