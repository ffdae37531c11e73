"""The continuous-batching driver's two schedules (slabs in input order, or
the first sweep of every slab and then the unsolved ones by decreasing
residual) give every slab the same sweeps, outcome and residual, bit for
bit: the batched kernels treat each problem of a launch alone, so the
composition of a round does not enter a slab's arithmetic.  Small heat slabs
of one grid with different parameters, fewer slots than slabs, the fallback
rule on (warm starts made by perturbing the plain ones)."""
import numpy as np
import pytest

import taps_workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[stream]", *a, flush=True)


@pytest.fixture(scope="module")
def env(taps_lib):
    import torch
    from paper_2503_13933_amd import capi, chain, warmstart
    h = capi.Handle()
    capi.taps_set_tuning(h, solver=capi.SOLVER_FAST_DIAG)
    yield torch, capi, chain, warmstart, h
    capi.taps_set_tuning(h, solver=capi.SOLVER_BLOCK_LU)
    h.close()


def _cases(n, seed, **grid):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [W.heat_slab(seed=seed * 7919 + i, power=float(rng.uniform(100, 300)), radius=float(rng.uniform(0.03, 0.08)),
                        k=float(rng.uniform(0.01, 0.03)), **grid) for i in range(n)]


def test_schedules_give_identical_slab_results(env):
    torch, capi, chain, ws, h = env
    grid = dict(nx=40, ny=36, nz=12, nt=25, M=10)
    n, slots, cap = 28, 8, 6
    cases = _cases(n, 11, **grid)
    probs = [chain.slab_problem(h, c) for c in cases]
    U0 = [W.initial_factors(c.axes, grid["M"], c.seed) for c in cases]
    plain = [torch.tensor(np.stack([u[d] for u in U0]), dtype=torch.float64, device="cuda") for d in range(4)]
    g = torch.Generator(device="cuda").manual_seed(5)
    warm = [t * (1.0 + 0.05 * torch.randn(t.shape, dtype=torch.float64, device="cuda", generator=g)) for t in plain]
    # the target: a residual some slabs reach after one sweep and some only later
    probe = ws.FactorBatch([t.clone() for t in plain])
    r = []
    for _ in range(3):
        _, rr = capi.taps_als_batched(h, [p.struct for p in probs], probe.ptrs(list(range(n))), 0.0, 1)
        r.append(rr)
    tol = float(np.nanmedian(r[2]))
    med1 = float(np.nanmedian(r[0]))
    res = {}
    for first in (False, True):
        U = ws.FactorBatch([t.clone() for t in warm])
        Up = ws.FactorBatch([t.clone() for t in plain])
        total, rho, restarts, outcome = ws.solve_stream(h, probs, U, tol, cap, slots, U_plain=Up, median_rho1=med1,
                                                        first_sweep_all=first)
        torch.cuda.synchronize()
        res[first] = (total, rho, restarts, outcome, [t.clone() for t in U.dims])
        _say(f"first_sweep_all={first}: sweeps {sorted(total)}, restarts {restarts}, outcomes {sorted(outcome)}")
    # the records packed once (as the benchmark passes them) give the same run
    U = ws.FactorBatch([t.clone() for t in warm])
    Up = ws.FactorBatch([t.clone() for t in plain])
    packed = ws.pack_problems(probs)
    c = ws.solve_stream(h, packed, U, tol, cap, slots, U_plain=Up, median_rho1=med1, first_sweep_all=True)
    torch.cuda.synchronize()
    assert c[0] == res[True][0] and c[3] == res[True][3]
    assert np.array_equal(np.asarray(c[1]), np.asarray(res[True][1]), equal_nan=True)
    for ta, tb in zip(U.dims, res[True][4]):
        assert torch.equal(ta, tb)
    a, b = res[False], res[True]
    assert a[0] == b[0] and a[2] == b[2] and a[3] == b[3]
    assert np.array_equal(np.asarray(a[1]), np.asarray(b[1]), equal_nan=True)
    for ta, tb in zip(a[4], b[4]):
        assert torch.equal(ta, tb)
    assert len(set(a[0])) > 1, "the case should mix slabs of different sweep counts"
