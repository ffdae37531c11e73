"""Batched Algorithm 1: every problem of a batch must give what the
single-problem path (and the oracle) gives on its own, including problems of
different grid sizes and problems that converge at different sweeps."""
import math

import numpy as np
import pytest

import parity_util as pu
import taps_workloads as W
from oracle import als, problems, separated

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


@pytest.fixture(scope="module")
def env(taps_lib):
    import torch
    from paper_2503_13933_amd import capi, problem
    h = capi.Handle()
    yield torch, capi, problem, h
    h.close()


@pytest.fixture(params=["blocklu", "fastdiag"])
def solver(env, request):
    torch, capi, problem, h = env
    capi.taps_set_tuning(h, solver=capi.SOLVER_FAST_DIAG if request.param == "fastdiag" else capi.SOLVER_BLOCK_LU)
    yield request.param
    capi.taps_set_tuning(h, solver=capi.SOLVER_BLOCK_LU)


def test_uneven_batch_matches_single_and_oracle(env, solver):
    torch, capi, problem, h = env
    cases = [W.heat_slab(40, 33, 10, 21, M=6, seed=11),
             W.heat_slab(67, 70, 13, 9, M=6, seed=12, power=120.0, radius=0.07),
             W.heat_slab(24, 20, 12, 17, M=6, seed=13, k=0.012, y0=0.35)]
    _say(f"batched: 3 uneven heat slabs, M=6, 2 sweeps ({solver})")
    devs = [problem.heat_slab(h, c) for c in cases]
    U0 = [W.initial_factors(c.axes, c.M, c.seed) for c in cases]
    Ub = [d.factors(u) for d, u in zip(devs, U0)]
    sweeps, rhos = capi.taps_als_batched(h, [d.struct for d in devs], Ub, 0.0, 2)
    torch.cuda.synchronize()
    assert sweeps == [2, 2, 2]
    for c, d, u0, ub, rb in zip(cases, devs, U0, Ub, rhos):
        Us = d.factors(u0)
        sw, rs, _ = capi.taps_als(h, d.struct, Us, 0.0, 2)
        torch.cuda.synchronize()
        ora = problems.heat_slab(c)
        Uo, rho_o, ch_o = pu.oracle_sweeps(ora, u0, 2)
        fbar, rbar, cbar, kappa = pu.sweep_bars(ora, u0, Uo, 2, rho_o[-1], ch_o[-1])
        ro = rho_o[-1]
        diffs = []
        for d, (a, b_, o) in enumerate(zip(ub, Us, Uo)):
            assert rel(a.cpu().numpy(), b_.cpu().numpy()) < 1e-12
            diffs.append(pu.check(a.cpu().numpy(), o, fbar[d], f"factor {d}"))
        assert abs(rb - rs) <= 1e-12 * rs
        assert abs(rb - ro) <= rbar
        _say(f"  n={[a.n for a in c.axes]} kappa {kappa:.1e} factor diffs {[f'{x:.1e}/{y:.1e}' for x, y in diffs]} "
             f"(bars {[f'{b:.0e}' for b in fbar]}); rho batched {rb:.6e} single {rs:.6e} oracle {ro:.6e}")


def test_batch_predicates_converged_problems(env, solver):
    # a rank-one manufactured heat field converges in a few sweeps; a Gaussian
    # slab with M = 1 needs many: each must stop at its own sweep count and
    # agree with its single-problem run
    torch, capi, problem, h = env
    cpoly = W.heat_slab(9, 8, 10, 7, M=1, seed=5)
    cgauss = W.heat_slab(24, 20, 12, 17, M=1, seed=7)
    _say(f"batched predication: polynomial + gaussian, M=1, tol 1e-10 ({solver})")
    dpoly = problem.heat_polynomial(h, cpoly)
    dg = problem.heat_slab(h, cgauss)
    u0 = [W.initial_factors(cpoly.axes, 1, 5), W.initial_factors(cgauss.axes, 1, 7)]
    Ub = [dpoly.factors(u0[0]), dg.factors(u0[1])]
    sweeps, rhos = capi.taps_als_batched(h, [dpoly.struct, dg.struct], Ub, 1e-10, 60)
    torch.cuda.synchronize()
    singles = []
    for d, u in zip([dpoly, dg], u0):
        U = d.factors(u)
        singles.append(capi.taps_als(h, d.struct, U, 1e-10, 60)[:2])
    _say(f"  batched sweeps {sweeps} rho {rhos}; single {singles}")
    assert sweeps[0] == singles[0][0] and sweeps[1] == singles[1][0]
    assert sweeps[0] < sweeps[1]
    for rb, (sw, rs) in zip(rhos, singles):
        assert abs(rb - rs) <= 1e-9 * rs + 1e-15


def test_batch_rejects_mismatched_modes(env):
    torch, capi, problem, h = env
    a = problem.heat_slab(h, W.heat_slab(8, 7, 6, 7, M=3))
    b = problem.heat_slab(h, W.heat_slab(8, 7, 6, 7, M=4))
    Ua = a.factors(W.initial_factors([x.ax for x in a.axes], 3, 1))
    Ub = b.factors(W.initial_factors([x.ax for x in b.axes], 4, 1))
    with pytest.raises(capi.TapsError):
        capi.taps_als_batched(h, [a.struct, b.struct], [Ua, Ub], 0.0, 1)


def test_profile_families_of_the_fast_diagonalisation(env):
    """Kernel timing: one batched sweep with the fast diagonalisation records
    one launch per dim in the banded-stage (solve), eigen-stage and real-Schur
    families, with the algorithmic work the C-ABI documents; the Schur kernel
    is timed inside the eigen-stage bracket, so its time is the smaller."""
    torch, capi, problem, h = env
    capi.taps_set_tuning(h, solver=capi.SOLVER_FAST_DIAG)
    try:
        cases = [W.heat_slab(40, 33, 10, 21, M=6, seed=21 + i) for i in range(3)]
        devs = [problem.heat_slab(h, c) for c in cases]
        Ub = [d.factors(W.initial_factors(c.axes, c.M, c.seed)) for c, d in zip(cases, devs)]
        torch.cuda.synchronize()
        capi.taps_profile_enable(h, True)
        capi.taps_als_batched(h, [d.struct for d in devs], Ub, 0.0, 1)
        torch.cuda.synchronize()
        capi.taps_profile_enable(h, False)
        D, M, B = 4, 6, len(cases)
        n_s, ms_s, fl_s, by_s = capi.taps_profile_read(h, capi.PROF_SOLVE)
        n_e, ms_e, fl_e, by_e = capi.taps_profile_read(h, capi.PROF_EIG)
        n_c, ms_c, fl_c, by_c = capi.taps_profile_read(h, capi.PROF_SCHUR)
        _say(f"profile: solve {n_s} x {ms_s:.3f} ms, eig {n_e} x {ms_e:.3f} ms, schur {n_c} x {ms_c:.3f} ms")
        assert n_s == n_e == n_c == D
        assert 0.0 < ms_c < ms_e
        assert fl_c == pytest.approx(D * B * 25.0 * M ** 3, rel=1e-12)
        assert by_c == pytest.approx(D * B * 24.0 * M ** 2, rel=1e-12)
        assert fl_e == pytest.approx(D * B * 44.0 * M ** 3, rel=1e-12)
        assert fl_s > 0.0 and by_s > 0.0
    finally:
        capi.taps_set_tuning(h, solver=capi.SOLVER_BLOCK_LU)


@pytest.mark.parametrize("M", [56, 60])
def test_batched_fast_diag_large_modes(env, M):
    """Fast diagonalisation at M above the common kernel layout (M <= 64
    layout; at M = 60 the complex Schur vectors go through the workspace),
    batched over two uneven slabs whose z and t dims have fewer rows than
    modes, one sweep against the oracle's."""
    torch, capi, problem, h = env
    cases = [W.heat_slab(70, 40, 15, 21, M=M, seed=21), W.heat_slab(52, 61, 9, 13, M=M, seed=22, k=0.015)]
    _say(f"batched fast diagonalisation, M={M}, slabs {[[a.n for a in c.axes] for c in cases]}")
    capi.taps_set_tuning(h, solver=capi.SOLVER_FAST_DIAG)
    try:
        devs = [problem.heat_slab(h, c) for c in cases]
        U0 = [W.initial_factors(c.axes, c.M, c.seed) for c in cases]
        Ub = [d.factors(u) for d, u in zip(devs, U0)]
        sweeps, rhos = capi.taps_als_batched(h, [d.struct for d in devs], Ub, 0.0, 1)
        torch.cuda.synchronize()
        assert sweeps == [1, 1]
        for c, u0, ub, rb in zip(cases, U0, Ub, rhos):
            ora = problems.heat_slab(c)
            Uo, rho_o, ch_o = pu.oracle_sweeps(ora, u0, 1)
            fbar, rbar, cbar, kappa = pu.sweep_bars(ora, u0, Uo, 1, rho_o[-1], ch_o[-1])
            diffs = [pu.check(a.cpu().numpy(), o, bar, f"factor {d}") for d, (a, o, bar) in enumerate(zip(ub, Uo, fbar))]
            assert abs(rb - rho_o[-1]) <= rbar
            _say(f"  kappa {kappa:.1e} factor diffs {[f'{x:.1e}/{y:.1e}' for x, y in diffs]} "
                 f"(bars {[f'{b:.0e}' for b in fbar]}); rho {rb:.8e} vs {rho_o[-1]:.8e}")
    finally:
        capi.taps_set_tuning(h, solver=capi.SOLVER_BLOCK_LU)
