"""Multi-slab space-time chains in the paper's multi-track regime (1.5 mm
cube, 5 um mesh, 200 W beam at 500 mm/s, Ti-6Al-4V): the chain driver
(carried initial condition as extra load terms, mode compression of the end
state) against the oracle on a small grid, and the study of how many time
points per slab pay (the paper finds about 20 best): a fixed stretch of scan
split into slabs of 5, 10 and 20 time steps, with the projected residual each
slab reaches."""
import time

import numpy as np
import pytest

import parity_util as pu
import taps_workloads as W
from oracle import chain as ochain
from oracle import fulltensor, problems

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[multitrack]", *a, flush=True)


@pytest.fixture(scope="module")
def env(taps_lib):
    import torch
    from paper_2503_13933_amd import capi, chain
    h = capi.Handle()
    capi.taps_set_tuning(h, solver=capi.SOLVER_FAST_DIAG)
    yield torch, capi, chain, h
    h.close()


def test_chain_of_multitrack_slabs_matches_oracle(env):
    torch, capi, chain, h = env
    cases = W.multitrack_slabs(10, 3, n=21, M=12)
    Kc = 4
    U0s = [W.initial_factors(c.axes, c.M, 60 + T) for T, c in enumerate(cases)]
    C0s = [W.initial_factors(c.axes[:3], Kc, 70 + T) for T, c in enumerate(cases)]
    _say("chain of 3 multi-track slabs 21^3 x 11, M=12, Kc=4: GPU vs oracle")
    dims = problems.dims_of(cases[0])
    ref = ochain.run_chain(cases, dims, U0s, C0s, sweeps=3, comp_sweeps=4)
    with pu.perturbed(1e-14, seed=3):
        pert = ochain.run_chain(cases, dims, U0s, C0s, sweeps=3, comp_sweeps=4)
    got = chain.run_chain(h, cases, U0s, C0s, sweeps=3, comp_sweeps=4)
    torch.cuda.synchronize()
    for T in range(3):
        fu = fulltensor.td_tensor(ref[T][0])
        bar = max(pu.TOL, 10 * pu.maxrel(fulltensor.td_tensor(pert[T][0]), fu))
        r = pu.check(fulltensor.td_tensor([u.cpu().numpy() for u in got[T][0]]), fu, bar, f"slab {T}")
        _say(f"  slab {T}: field rel/max {r[0]:.1e}/{r[1]:.1e} (bar {bar:.0e})")


@pytest.mark.timeout(900)
def test_time_points_per_slab_study(env):
    torch, capi, chain, h = env
    steps_total, Kc = 80, 10
    for steps in (5, 10, 20):
        cases = W.multitrack_slabs(steps, steps_total // steps, n=301)
        M = cases[0].M
        V = None
        rhos, chgs = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for T, c in enumerate(cases):
            prob = chain.slab_problem(h, c, V)
            U = prob.factors(W.initial_factors(c.axes, M, c.seed))
            ch = []
            _, rho, _ = capi.taps_als(h, prob.struct, U, 0.0, 3, change_hist=ch)
            rhos.append(rho)
            chgs.append(ch[-1])
            comp = chain.compression_problem(h, prob, V, U, Kc)
            Vn = comp.factors(W.initial_factors(c.axes[:3], Kc, c.seed + 1))
            capi.taps_als(h, comp.struct, Vn, 0.0, 4)
            V = Vn
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        # how far Algorithm 1 gets on one slab of this length
        c = cases[1]
        prob = chain.slab_problem(h, c, None)
        U = prob.factors(W.initial_factors(c.axes, M, c.seed))
        _, rho30, hist = capi.taps_als(h, prob.struct, U, 0.0, 30)
        best = np.nanmin(hist)
        _say(f"  {steps} steps per slab (M={M}), {len(cases)} slabs for {steps_total} steps of scan: {el:.2f} s "
             f"({el / len(cases) * 1e3:.1f} ms per slab, {el / (steps_total * 0.01):.2f} s per ms of scan); "
             f"rho after 3 sweeps median {np.nanmedian(rhos):.2e}, change {np.nanmedian(chgs):.2e}; "
             f"30 sweeps on one slab: best rho {best:.2e}, last {hist[-1]:.2e}")
        assert len(rhos) == len(cases)
