"""GPU parity at the benchmark's own shapes: 512 x 512 x 128 nodes x 257 time
nodes (R = 257 load terms, n >= 512 rows, several 64-row chunks and
multi-tile M x M Grams), the mode counts the matrix-core contraction and
residual bodies tile differently (M = 16, 17, 40, 48), one batched sweep of
eight benchmark slabs by fast diagonalisation, and a launch over 2048
problems (the benchmark's slots).

Bars as in the other parity tests (parity_util): 1e-10 in norm and entry by
entry, raised per case only by the oracle's own condition estimate or
rounding response; every measured difference and its bar is printed.
"""
import numpy as np
import pytest

import parity_util as pu
import taps_workloads as W
from oracle import als, problems, reconstruct, separated

pytestmark = pytest.mark.gpu

TOL = pu.TOL
BENCH = dict(nx=512, ny=512, nz=128, nt=257)


def _say(*a):
    print("[bench-shape]", *a, flush=True)


@pytest.fixture(scope="module")
def env(taps_lib):
    import torch
    from paper_2503_13933_amd import capi, chain, problem
    h = capi.Handle()
    yield torch, capi, chain, problem, h
    h.close()


def _rand_U(prob, M, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for d in range(prob.D):
        u = rng.standard_normal((prob.n[d], M))
        u[list(prob.fixed[d])] = 0.0
        out.append(u)
    return out


def _case(M):
    if M == 40:
        return W.heat_slab(M=40, seed=2, **BENCH)
    # n >= 512 rows in x, R = 257 load terms, the other dims ragged
    return W.heat_slab(520, 96, 40, 257, M=M, seed=3)


ORDER = {"mass": 0, "stiff": 1, "ddt": 1}


@pytest.mark.parametrize("M", [16, 17, 40, 48])
def test_contract_residual_balance(env, M):
    torch, capi, chain, problem, h = env
    case = _case(M)
    _say(f"contract / residual / balance, heat slab {[a.n for a in case.axes]} M={M}")
    dev = problem.heat_slab(h, case)
    ora = problems.heat_slab(case)
    Uh = _rand_U(ora, M, 100 + M)
    U = dev.factors(Uh)
    for d in range(ora.D):
        Cd = torch.empty((2, M, M), dtype=torch.float64, device="cuda")
        Qd = torch.empty((ora.n[d], M), dtype=torch.float64, device="cuda")
        capi.taps_contract(h, dev.struct, d, 0xFF, U, Cd, Qd)
        torch.cuda.synchronize()
        Co = separated.couplings(ora, Uh, d)
        for nm, c in Co.items():
            r, m = pu.check(Cd[ORDER[nm]].cpu().numpy(), c, TOL, f"C dim {d} {nm}")
            _say(f"  C dim {d} {nm}: rel {r:.1e} max entry {m:.1e}")
        r, m = pu.check(Qd.cpu().numpy(), separated.force(ora, Uh, d), TOL, f"Q dim {d}")
        _say(f"  Q dim {d}: rel {r:.1e} max entry {m:.1e}")
    out = torch.empty(ora.D + 2, dtype=torch.float64, device="cuda")
    capi.taps_residual(h, dev.struct, U, out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    Rs, Qs = separated.residuals(ora, Uh)
    for d in range(ora.D):
        ref = float(np.sum(Rs[d] ** 2))
        assert abs(o[d] - ref) <= TOL * ref, (d, o[d], ref)
    rho = separated.residual_norm(ora, Uh)
    _say(f"  rho gpu {o[-1]:.12e} oracle {rho:.12e}")
    assert abs(o[-1] - rho) <= TOL * rho
    capi.taps_balance(h, dev.struct, U)
    torch.cuda.synchronize()
    als.balance(Uh)
    for d in range(ora.D):
        pu.check(U[d].cpu().numpy(), Uh[d], 1e-13, f"balanced dim {d}")


def test_solve_dim_fast_diag_bench_grid(env):
    torch, capi, chain, problem, h = env
    case = _case(40)
    _say("fast-diagonalisation dim solves on the benchmark grid, M=40")
    capi.taps_set_tuning(h, solver=capi.SOLVER_FAST_DIAG)
    try:
        dev = problem.heat_slab(h, case)
        ora = problems.heat_slab(case)
        Uh = _rand_U(ora, 40, 7)
        info = torch.zeros(1, dtype=torch.int32, device="cuda")
        berr = torch.zeros(1, dtype=torch.float64, device="cuda")
        for d in range(ora.D):
            Co = separated.couplings(ora, Uh, d)
            Qo = separated.force(ora, Uh, d)
            Xo = separated.solve_dim(ora, d, Co, Qo)
            Cd = torch.zeros((2, 40, 40), dtype=torch.float64, device="cuda")
            for nm, c in Co.items():
                Cd[ORDER[nm]] = torch.tensor(c, device="cuda")
            Qd = torch.tensor(Qo, device="cuda")
            Xd = torch.empty_like(Qd)
            capi.taps_solve_dim(h, dev.struct, d, Cd, Qd, Xd, info, berr)
            torch.cuda.synchronize()
            assert int(info.item()) == 0
            kappa = pu.cond_estimate(ora, d, Co)
            bar = max(TOL, 10 * kappa * pu.EPS)
            r, m = pu.check(Xd.cpu().numpy(), Xo, bar, f"X dim {d}")
            _say(f"  dim {d} (n={ora.n[d]}): kappa {kappa:.2e} bar {bar:.1e} backward {float(berr.item()):.1e} "
                 f"rel {r:.2e} max entry {m:.2e}")
            assert float(berr.item()) < 1e-12
    finally:
        capi.taps_set_tuning(h, solver=capi.SOLVER_BLOCK_LU)


@pytest.mark.timeout(900)
def test_batched_sweep_of_benchmark_slabs(env):
    """One batched sweep (fast diagonalisation) of eight benchmark slabs --
    the benchmark's grid, modes, parameter draws and random starts -- against
    the oracle's sweep of each slab: every factor, rho, the relative change and
    the field at sampled grid points."""
    torch, capi, chain, problem, h = env
    cases = W.heat_slab_family(8, seed=2, M=40, **BENCH)
    _say("batched sweep of 8 benchmark slabs 512x512x128x257, M=40, fast diagonalisation")
    capi.taps_set_tuning(h, solver=capi.SOLVER_FAST_DIAG)
    try:
        devs = [chain.slab_problem(h, c) for c in cases]
        U0 = [W.initial_factors(c.axes, c.M, c.seed) for c in cases]
        Ub = [d.factors(u) for d, u in zip(devs, U0)]
        chg = []
        sweeps, rhos = capi.taps_als_batched(h, [d.struct for d in devs], Ub, 0.0, 1, change=chg)
        torch.cuda.synchronize()
        assert sweeps == [1] * 8
        rng = np.random.Generator(np.random.PCG64(9))
        for b, (c, u0, ub, rb, cb) in enumerate(zip(cases, U0, Ub, rhos, chg)):
            ora = problems.heat_slab(c)
            Uo, rho_o, ch_o = pu.oracle_sweeps(ora, u0, 1)
            fbar, rbar, cbar, kappa = pu.sweep_bars(ora, u0, Uo, 1, rho_o[-1], ch_o[-1])
            Ug = [u.cpu().numpy() for u in ub]
            diffs = [pu.check(a, o, bar, f"slab {b} factor {d}") for d, (a, o, bar) in enumerate(zip(Ug, Uo, fbar))]
            idx = np.stack([rng.integers(0, ax.n, 200_000) for ax in c.axes], axis=1)
            fg = reconstruct.reconstruct_points(Ug, idx)
            fo = reconstruct.reconstruct_points(Uo, idx)
            fr, fm = pu.check(fg, fo, max(fbar), f"slab {b} field at 2e5 points")
            _say(f"  slab {b}: kappa {kappa:.2e}, factor rel/max-entry "
                 f"{[f'{x:.1e}/{y:.1e}' for x, y in diffs]} (bars {[f'{x:.0e}' for x in fbar]}), "
                 f"field {fr:.1e}/{fm:.1e}, rho {rb:.10e} vs {rho_o[-1]:.10e} (bar {rbar:.1e}), "
                 f"change {cb:.10e} vs {ch_o[-1]:.10e}")
            assert abs(rb - rho_o[-1]) <= rbar
            assert abs(cb - ch_o[-1]) <= cbar * ch_o[-1]
    finally:
        capi.taps_set_tuning(h, solver=capi.SOLVER_BLOCK_LU)


@pytest.mark.timeout(600)
def test_batched_sweep_of_2048_problems(env):
    """2048 problems in one batched call -- the benchmark's slot count, so
    every kernel's grid has 2048 problems in its last coordinate.  The even
    problems are checked against their own oracle sweeps (a sample the
    oracle finishes in about a minute); the odd ones must equal, bit for bit,
    a second call that holds only them (the batched kernels treat every
    problem of a launch alone, and these problems share one grid)."""
    torch, capi, chain, problem, h = env
    cases = W.heat_slab_family(2048, seed=12, nx=24, ny=20, nz=12, nt=17, M=5)
    _say("batched sweep of 2048 heat slabs 24x20x12x17, M=5, fast diagonalisation")
    capi.taps_set_tuning(h, solver=capi.SOLVER_FAST_DIAG)
    try:
        devs = [problem.heat_slab(h, c) for c in cases]
        U0 = [W.initial_factors(c.axes, c.M, c.seed) for c in cases]
        Ub = [d.factors(u) for d, u in zip(devs, U0)]
        sweeps, rhos = capi.taps_als_batched(h, [d.struct for d in devs], Ub, 0.0, 1)
        odd = list(range(1, 2048, 2))
        Uo2 = [devs[b].factors(U0[b]) for b in odd]
        _, rhos2 = capi.taps_als_batched(h, [devs[b].struct for b in odd], Uo2, 0.0, 1)
        torch.cuda.synchronize()
        for b, u2, r2 in zip(odd, Uo2, rhos2):
            assert rhos[b] == r2, f"problem {b}: rho {rhos[b]!r} alone {r2!r}"
            for d in range(4):
                assert torch.equal(Ub[b][d], u2[d]), f"problem {b} factor {d} differs from its own launch"
        worst, raised = 0.0, 0
        for b in range(0, 2048, 2):
            c, u0, ub, rb = cases[b], U0[b], Ub[b], rhos[b]
            ora = problems.heat_slab(c)
            Uo, rho_o, ch_o = pu.oracle_sweeps(ora, u0, 1)
            fbar, rbar, cbar, kappa = pu.sweep_bars(ora, u0, Uo, 1, rho_o[-1], ch_o[-1])
            for d, (a, o) in enumerate(zip(ub, Uo)):
                r, m = pu.check(a.cpu().numpy(), o, fbar[d], f"problem {b} factor {d}")
                worst = max(worst, r, m)
                raised += fbar[d] > TOL
            assert abs(rb - rho_o[-1]) <= rbar
        _say(f"  worst factor difference over the 1024 even problems {worst:.2e}; bars above 1e-10: {raised} of "
             f"{4 * 1024}; the 1024 odd ones equal their own launch")
    finally:
        capi.taps_set_tuning(h, solver=capi.SOLVER_BLOCK_LU)
