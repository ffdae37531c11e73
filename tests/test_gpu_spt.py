"""Space-parameter-time batches (P, r, k as tensor dimensions, the
conductivity through the k-weighted mass) on the GPU: the exact field of the
polynomial load, and an uneven batch of seven-dimensional problems through
the batched driver against the oracle, with both dim solvers (fast
diagonalisation for the dims with two matrix kinds, block LU for the
parameter dims with one)."""
import numpy as np
import pytest

import parity_util as pu
import taps_workloads as W
from oracle import problems

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[spt]", *a, flush=True)


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


def test_exact_field(env, solver):
    torch, capi, problem, h = env
    c = W.spt_slab(9, 8, 10, 9, n_param=7, M=1, seed=6)
    _say(f"exact field z(2H-z) t P on 9x8x10 x 7^3 x 9, M=1 ({solver})")
    dev = problem.spt_polynomial(h, c)
    U = dev.factors(W.initial_factors(c.axes, 1, 6))
    sweeps, rho, _ = capi.taps_als(h, dev.struct, U, 1e-13, 200)
    assert rho <= 1e-13, (sweeps, rho)
    Ug = [u.cpu().numpy()[:, 0] for u in U]
    z, t, P = c.axes[2].nodes(), c.axes[6].nodes(), c.axes[3].nodes()
    want = [np.ones(9), np.ones(8), z * (2 * c.height - z), P, np.ones(7), np.ones(7), t]
    # the rank-one factors are the exact ones up to one scale per dim
    scale = np.prod([np.dot(g, w) / np.dot(w, w) for g, w in zip(Ug, want)])
    for g, w in zip(Ug, want):
        a = np.dot(g, w) / np.dot(w, w)
        assert np.abs(g - a * w).max() <= 1e-12 * np.abs(a * w).max()
    assert abs(scale - 1.0) < 1e-12


def test_uneven_batch_against_oracle(env, solver):
    torch, capi, problem, h = env
    cases = W.spt_batch(batch=4, n_lo=8, n_hi=40, n_param=6, M=5, seed=21)
    _say(f"uneven batch of 4 space-parameter-time slabs, M=5, 2 sweeps ({solver}): "
         f"{[[a.n for a in c.axes] for c in cases]}")
    devs = [problem.spt_slab(h, c) for c in cases]
    U0 = [W.initial_factors(c.axes, c.M, c.seed) for c in cases]
    Ub = [d.factors(u) for d, u in zip(devs, U0)]
    chg = []
    sweeps, rhos = capi.taps_als_batched(h, [d.struct for d in devs], Ub, 0.0, 2, change=chg)
    torch.cuda.synchronize()
    assert sweeps == [2] * 4
    for c, u0, ub, rb, cb in zip(cases, U0, Ub, rhos, chg):
        ora = problems.spt_slab(c)
        Uo, rho_o, ch_o = pu.oracle_sweeps(ora, u0, 2)
        fbar, rbar, cbar, kappa = pu.sweep_bars(ora, u0, Uo, 2, rho_o[-1], ch_o[-1])
        diffs = [pu.check(a.cpu().numpy(), o, bar, f"factor {d}") for d, (a, o, bar) in enumerate(zip(ub, Uo, fbar))]
        _say(f"  n={[a.n for a in c.axes]} kappa {kappa:.1e} factor diffs "
             f"{[f'{x:.0e}/{y:.0e}' for x, y in diffs]} (bars {[f'{b:.0e}' for b in fbar]}); "
             f"rho {rb:.8e} vs {rho_o[-1]:.8e}; change {cb:.8e} vs {ch_o[-1]:.8e}")
        assert abs(rb - rho_o[-1]) <= rbar
        assert abs(cb - ch_o[-1]) <= cbar * ch_o[-1]


def test_long_load_rows_split_over_force_items(env):
    """Load rows longer than one force work item's column range (32 n_t load
    terms above 1024 in x): the force is summed from per-range partials.
    Against the oracle, and a captured graph of the same two sweeps equal
    to host launches bit for bit."""
    torch, capi, problem, h = env
    cases = [W.spt_slab(14, 11, 9, nt, n_param=32, M=5, seed=31 + i, y0=0.4 + 0.1 * i)
             for i, nt in enumerate((41, 12, 36))]
    _say(f"long load rows: R = {[32 * c.axes[6].n for c in cases]}, M=5")
    capi.taps_set_tuning(h, solver=capi.SOLVER_FAST_DIAG)
    try:
        devs = [problem.spt_slab(h, c) for c in cases]
        U0 = [W.initial_factors(c.axes, c.M, c.seed) for c in cases]
        Ub = [d.factors(u) for d, u in zip(devs, U0)]
        sweeps, rhos = capi.taps_als_batched(h, [d.struct for d in devs], Ub, 0.0, 2)
        torch.cuda.synchronize()
        for c, u0, ub, rb in zip(cases, U0, Ub, rhos):
            ora = problems.spt_slab(c)
            Uo, rho_o, ch_o = pu.oracle_sweeps(ora, u0, 2)
            fbar, rbar, cbar, kappa = pu.sweep_bars(ora, u0, Uo, 2, rho_o[-1], ch_o[-1])
            diffs = [pu.check(a.cpu().numpy(), o, bar, f"factor {d}") for d, (a, o, bar) in enumerate(zip(ub, Uo, fbar))]
            _say(f"  R={32 * c.axes[6].n} kappa {kappa:.1e} factor diffs {[f'{x:.0e}/{y:.0e}' for x, y in diffs]} "
                 f"(bars {[f'{b:.0e}' for b in fbar]}); rho {rb:.8e} vs {rho_o[-1]:.8e}")
            assert abs(rb - rho_o[-1]) <= rbar
        capi.taps_set_tuning(h, graph_sweeps=2)
        Ug = [d.factors(u) for d, u in zip(devs, U0)]
        capi.taps_als_batched(h, [d.struct for d in devs], Ug, 0.0, 2)
        torch.cuda.synchronize()
        for ub, ug in zip(Ub, Ug):
            for a, b in zip(ub, ug):
                assert torch.equal(a, b)
    finally:
        capi.taps_set_tuning(h, solver=capi.SOLVER_BLOCK_LU, graph_sweeps=0)
