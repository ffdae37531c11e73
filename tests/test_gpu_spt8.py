"""The eight-dimensional space-parameter-time convergence study of the
paper's second results section on the GPU (x, y, z, k, P, rho, c_p, t):
the problem the library builds (derived source, nodal lifting, the k, rho
and c_p weighted masses) against the oracle's, and the relative L2 error
against the closed-form field under simultaneous refinement of every dim
up to 450 nodes (the paper's largest grid, 450^8 ~ 1.7e21 equivalent
unknowns)."""
import time

import numpy as np
import pytest

import parity_util as pu
import st_error
import taps_workloads as W
from oracle import problems

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[spt8]", *a, flush=True)


@pytest.fixture(scope="module")
def env(taps_lib):
    import torch
    from paper_2503_13933_amd import capi, problem
    h = capi.Handle()
    capi.taps_set_tuning(h, solver=capi.SOLVER_FAST_DIAG)
    yield torch, capi, problem, h
    h.close()


def test_problem_and_sweeps_match_oracle(env):
    torch, capi, problem, h = env
    c = W.spt8_convergence(7, M=4)
    _say("eight dims 7^8, M=4: 2 sweeps against the oracle")
    dev = problem.spt8_convergence(h, c)
    dims = problems.dims_of(c)
    ora = problems.spt8_convergence(c, dims)
    U0 = W.initial_factors(c.axes, c.M, c.seed)
    U = dev.factors(U0)
    chg = []
    sweeps, rho, _ = capi.taps_als(h, dev.struct, U, 0.0, 2, change_hist=chg)
    Uo, rho_o, ch_o = pu.oracle_sweeps(ora, U0, 2)
    fbar, rbar, cbar, kappa = pu.sweep_bars(ora, U0, Uo, 2, rho_o[-1], ch_o[-1])
    Ug = [u.cpu().numpy() for u in U]
    diffs = [pu.check(a, o, bar, f"factor {d}") for d, (a, o, bar) in enumerate(zip(Ug, Uo, fbar))]
    _say(f"  kappa {kappa:.1e}, factor diffs {[f'{x:.0e}/{y:.0e}' for x, y in diffs]}, "
         f"rho {rho:.8e} vs {rho_o[-1]:.8e}")
    assert abs(rho - rho_o[-1]) <= rbar
    assert abs(chg[-1] - ch_o[-1]) <= cbar * ch_o[-1]
    full = [f.cpu().numpy() for f in dev.full_factors(U)]
    ref = problems.spt8_field_factors(c, dims, Uo)
    e_g, e_o = st_error.spt8_l2_error(c, dims, full), st_error.spt8_l2_error(c, dims, ref)
    _say(f"  L2 error gpu {e_g:.10e} oracle {e_o:.10e}")
    assert abs(e_g - e_o) <= max(fbar) * 10 * max(1.0, 1.0 / e_o)


@pytest.mark.timeout(900)
def test_convergence_to_450_nodes(env):
    torch, capi, problem, h = env
    for s, p, ns in ((1, 1, (10, 20, 40, 80, 160, 320, 450)), (2, 2, (10, 20, 40, 80, 160))):
        errs = []
        for n in ns:
            c = W.spt8_convergence(n, M=12, s=s, p=p)
            dims = problems.dims_of(c)
            dev = problem.spt8_convergence(h, c)
            U = dev.factors(W.initial_factors(c.axes, c.M, c.seed))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sweeps, rho, _ = capi.taps_als(h, dev.struct, U, 0.0, 4)
            note = "" if rho == rho else f" (stopped after sweep {sweeps}: {capi.last_error(h)})"
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            e = st_error.spt8_l2_error(c, dims, [f.cpu().numpy() for f in dev.full_factors(U)])
            rate = np.log(errs[-1] / e) / np.log(n / ns[len(errs) - 1]) if errs else float("nan")
            errs.append(e)
            _say(f"  s={s} p={p} {n}^8 ({float(n) ** 8:.2e} equivalent unknowns), M=12, 4 sweeps in {el:.2f} s: "
                 f"L2 error {e:.3e}, rate {rate:.2f}, rho {rho:.2e}{note}")
        assert errs[1] < errs[0] and errs[3] < errs[2]
