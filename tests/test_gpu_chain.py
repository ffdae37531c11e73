"""Slab chain on the GPU against the chain oracle: carried initial condition
as extra load terms, mode compression by Algorithm 1 on the mass operator,
both driven through the C ABI (taps_band_apply, taps_als)."""
import numpy as np
import pytest

import parity_util as pu
import taps_workloads as W
from oracle import chain as ochain
from oracle import fulltensor, problems
from oracle.assemble import Dim1D

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[chain]", *a, flush=True)


@pytest.fixture(scope="module")
def env(taps_lib):
    import torch
    from paper_2503_13933_amd import capi, chain
    h = capi.Handle()
    yield torch, capi, chain, h
    h.close()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("s", [1, 2])
def test_band_apply_matches_matrices(env, s):
    torch, capi, chain, h = env
    _say(f"band apply s={s}")
    ax = W.Axis("x", 0.0, 1.3, 37, s, 20.0, min(s, 2), 5)
    from paper_2503_13933_amd.problem import DeviceAxis
    A = DeviceAxis(h, ax, [capi.MASS, capi.STIFF], "cuda").assemble(
        torch.zeros((1, (ax.n - 1) * ax.n_gauss), dtype=torch.float64, device="cuda"))
    d = Dim1D(ax.nodes(), s, 20.0, min(s, 2), 5)
    rng = np.random.Generator(np.random.PCG64(s))
    X = rng.standard_normal((37, 9))
    sc = rng.standard_normal(5)
    dX = torch.tensor(X, device="cuda")
    wide = torch.zeros((37, 12), dtype=torch.float64, device="cuda")
    capi.taps_band_apply(h, s, A.band[1], dX[:, 2:7], wide[:, 3:8], alpha=-0.7,
                         scale=torch.tensor(sc, device="cuda"))
    got = wide.cpu().numpy()
    ref = -0.7 * (d.matrix("stiff") @ X[:, 2:7]) * sc[None, :]
    assert rel(got[:, 3:8], ref) < 1e-13
    assert np.all(got[:, :3] == 0) and np.all(got[:, 8:] == 0)


def test_chain_matches_oracle(env):
    torch, capi, chain, h = env
    base = W.heat_slab(20, 16, 9, 9, M=4, seed=0, s=1, p=1)
    cases = [W.replace(base, x_start=0.1 + 0.25 * T, power=150.0 + 40.0 * T) for T in range(3)]
    Kc = 3
    U0s = [W.initial_factors(c.axes, c.M, 30 + T) for T, c in enumerate(cases)]
    C0s = [W.initial_factors(c.axes[:3], Kc, 40 + T) for T, c in enumerate(cases)]
    _say("chain 3 slabs 20x16x9x9 M=4 Kc=3 on the oracle")
    dims = problems.dims_of(base)
    ref = ochain.run_chain(cases, dims, U0s, C0s, sweeps=4, comp_sweeps=4)
    # the chain's own rounding amplification: the same chain with every dim
    # solve's couplings and force perturbed by 1e-14 of their RMS entry
    with pu.perturbed(1e-14, seed=1):
        pert = ochain.run_chain(cases, dims, U0s, C0s, sweeps=4, comp_sweeps=4)
    _say("chain on the GPU")
    got = chain.run_chain(h, cases, U0s, C0s, sweeps=4, comp_sweeps=4)
    torch.cuda.synchronize()
    for T in range(3):
        Ug = [u.cpu().numpy() for u in got[T][0]]
        Vg = [v.cpu().numpy() for v in got[T][2]]
        fu, fv = fulltensor.td_tensor(ref[T][0]), fulltensor.td_tensor(ref[T][2])
        bar_u = max(pu.TOL, 10 * pu.rel(fulltensor.td_tensor(pert[T][0]), fu),
                    10 * pu.maxrel(fulltensor.td_tensor(pert[T][0]), fu))
        bar_v = max(pu.TOL, 10 * pu.rel(fulltensor.td_tensor(pert[T][2]), fv),
                    10 * pu.maxrel(fulltensor.td_tensor(pert[T][2]), fv))
        e_u = pu.check(fulltensor.td_tensor(Ug), fu, bar_u, f"slab {T} field")
        e_v = pu.check(fulltensor.td_tensor(Vg), fv, bar_v, f"slab {T} carried field")
        _say(f"  slab {T}: slab field rel/max {e_u[0]:.2e}/{e_u[1]:.2e} (bar {bar_u:.1e}), "
             f"carried field {e_v[0]:.2e}/{e_v[1]:.2e} (bar {bar_v:.1e})")
        assert np.all(Vg[2][0] == 0.0)
